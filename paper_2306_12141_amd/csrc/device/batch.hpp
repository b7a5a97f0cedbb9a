// Device-side layout of a batched decode (many independent streams, one launch).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "decode.hpp"

namespace recoil {

// One stream of the batch. Offsets are bytes from the workspace base (words,
// table, unit records, lane records) or from the output base (out).
struct StreamDesc {
    uint64_t words_off, lut_off, meta_off, lanes_off, out_off;
    uint64_t n_symbols;
    uint32_t units;
    uint8_t quant_bits, symbol_bytes, lanes, single_symbol;
    uint32_t fill_symbol;
    uint16_t partitioned;   // conventional sub-sequences (see DecodeParams::partitioned)
    uint16_t lut_chunks;    // decode-table size in 16-byte chunks
};
static_assert(sizeof(StreamDesc) == 64, "StreamDesc is 64 bytes");

// Consecutive pairs of one stream, decoded by one workgroup. The stream's
// units are decoded in runs of `run` consecutive units (Sec. 3.3; 0 or 1: every
// split point), and a pair is two runs (W = 32) or one (W = 64, or W = 32 with
// kItemSingle set in `run`: one unit per wave, the upper half-wave idle, for a
// stream with no more runs than a workgroup has waves).
struct WorkItem {
    uint32_t stream;
    uint32_t first;     // first pair
    uint32_t count;
    uint32_t run;       // units per run, | kItemSingle
};
constexpr uint32_t kItemSingle = 0x80000000u;

struct BatchParams {
    const unsigned char *ws;      // workspace base
    uint32_t wide;                // nonzero: the two-level tables of 13 <= n <= 16 (a kernel of their own)
    unsigned char *out;           // output base
    const StreamDesc *streams;
    const WorkItem *items;
    uint32_t *head;               // work-queue head (device counter, reset before each launch)
    uint32_t *err;                // error word(s): err[stream * err_stride]
    uint32_t n_items;
    uint32_t lut_bytes;           // LDS bytes reserved for the largest table in the batch
    uint32_t err_stride;          // 0: one error word for the launch; 1: one per stream
    // Per-stream completion (both NULL to disable): remaining[s] counts the
    // stream's items not yet finished; the workgroup that finishes the last one
    // stores kHostDone | error bits to host_done[s] (host-visible memory).
    uint32_t *remaining;
    uint32_t *host_done;
};
constexpr uint32_t kHostDone = 0x80000000u;

struct BatchTuning {
    uint32_t waves;       // waves per workgroup: 8 or 16
    uint32_t chunk_groups;// K: groups per super-step (ring chunk = K*W words): 4 or 8
    uint32_t blocks_per_cu;// 0: occupancy limit
};

// Statically allocated queue heads (recoil_decode_batch_noalloc): one device
// array per GPU of kStaticScratchWords words, a head every kStaticHeadStride words.
constexpr uint32_t kStaticScratchWords = 96, kStaticHeadStride = 32;
// Device address of that array on the current device, looked up once per device.
hipError_t static_scratch(uint32_t **ptr);

// Persistent batched launch: queue-head reset kernel + decode kernel on `stream`.
hipError_t launch_batch(const BatchParams &bp, const BatchTuning &t, hipStream_t stream);
// Occupancy-derived workgroups per CU for a tuning (0 if the tuning is not available),
// of the kernel for one-level tables or, with wide set, for two-level ones.
int batch_blocks_per_cu(const BatchTuning &t, uint32_t lut_bytes, bool wide = false);

}  // namespace recoil
