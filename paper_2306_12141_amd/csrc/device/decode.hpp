// Device-side layout shared by the host planner and the HIP kernels.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace recoil {

// Per decode unit (0-based u; unit u starts at split point u+1, the last unit
// at the final states). Symbol groups are 0-based.
struct UnitMeta {
    uint32_t next;   // words available: the unit's first read is words[next - 1]
    uint32_t top;    // first group decoded (the anchor; G-1 for the last unit)
    uint32_t ghi;    // highest group whose symbols this unit stores
    uint32_t glo;    // lowest group decoded and stored
};

// Per lane of a unit: recorded state (bits 0..15) and activation step
// (bits 16..31) = top - group of the lane's recorded symbol. For the last unit
// the word is the full 32-bit final state and every lane is active at once.
//
// Decode table entries, indexed by slot = x mod 2^n (n <= 12):
//   8-bit symbols:  bits 0..7 symbol, 8..19 f(s), 20..31 slot - F(s)     (f < 4096)
//   16-bit symbols: .x = f(s) | (slot - F(s)) << 16, .y = symbol
// Wide tables (13 <= n <= 16, either symbol size), in two levels so that they fit
// LDS: 2^(n-4) bucket words, then one u32x2 per symbol with f > 0 in symbol
// order (its rank r). Bucket word b covers slots 16b .. 16b+15: bits 16..31 the
// rank of the symbol holding slot 16b, bit i-1 (i = 1..15) set when a symbol's
// range starts at slot 16b + i. Rank entry: .x = f(s), .y = s | F(s) << 16.
//
// The words array handed to the kernels is readable (padding) up to the next
// multiple of kChunkPadWords past B, because bitstream chunks are fetched whole.
constexpr uint32_t kChunkPadWords = 1024;

// Largest decode table staged in LDS (adaptive tables, wide tables).
constexpr uint32_t kMaxTableBytes = 65536;

struct DecodeParams {
    const uint16_t *words;      // B words (+ padding, see above)
    const void *lut;            // 2^n entries
    const UnitMeta *meta;       // M
    const uint32_t *lanes;      // M x W
    void *out;                  // N symbols
    uint32_t *err;              // device error word
    uint32_t *counts;           // checking launches only: N per-symbol store counts (else NULL)
    const uint8_t *tidx;        // adaptive coding: N per-symbol table indices (else NULL)
    uint32_t tables;            // decode tables in lut (1 unless adaptive)
    uint32_t lut_bytes;         // bytes of lut staged in LDS (a multiple of 16)
    uint64_t n_symbols;
    uint32_t units;
    uint32_t run;               // consecutive units decoded as one (Sec. 3.3): 1 uses every split point
    uint32_t runs;              // ceil(units / run); run r covers units [r run, min((r + 1) run, units))
    uint32_t quant_bits;
    uint32_t fill_symbol;       // used when the table holds a single symbol (f = 2^n)
    uint32_t single_symbol;     // nonzero: the stream is one repeated symbol
    uint32_t partitioned;       // nonzero: conventional sub-sequences (Sec. 2.3): every unit starts
                                // from its own 32-bit final states, no synchronisation, no run-on
};

// Launch shape of the single-stream kernel: waves per workgroup (1, 8 or 16;
// 0 = 16, or 1 when the launch has no more waves of work than the chip has
// SIMDs, or 8 when 16-wave workgroups would not reach every CU), groups per
// super-step K (4 or 8), workgroups per CU cap (0 =
// occupancy limit), units per run (0 = chosen from the number of resident waves).
struct DecodeTuning {
    uint32_t waves = 0, chunk_groups = 4, blocks_per_cu = 0, units_per_run = 0;
};

// Units per run when the tuning leaves it open: ceil(units / slots), so that
// every unit slot of the resident grid (resident waves x units per wave) decodes
// at most one run. Fewer, longer runs pay a unit's fixed costs less often, and
// with one run per slot no wave holds a second run that others wait for.
inline uint32_t auto_units_per_run(uint32_t units, uint64_t slots) {
    const uint64_t k = slots ? (units + slots - 1) / slots : 1;
    return k < 1 ? 1u : (uint32_t)k;
}

// Grid of a single-stream launch and the runs it decodes.
struct DecodeShape {
    uint32_t blocks, waves, units_per_run, runs, units_per_wave;
};

// Compute units of the current device (at least 1), cached per device.
int device_cus();

// Launcher (decode.hip). Returns hipSuccess or the launch error. With shape
// non-null nothing is launched: the grid and runs a launch would use are
// stored there (all zero when no decode kernel would run).
hipError_t launch_decode(const DecodeParams &p, uint32_t lanes, uint32_t symbol_bytes, const DecodeTuning &t,
                         hipStream_t stream, DecodeShape *shape = nullptr);

}  // namespace recoil
