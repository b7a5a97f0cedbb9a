// Recoil split decoding on gfx950 (Lin et al., ICPP 2023, Sec. 4.1).
//
// Mapping. A decode unit is W interleaved rANS lanes; one 64-lane wavefront
// runs one unit (W = 64) or two (W = 32, one per half-wave). Lane j of a unit
// keeps coder j's 32-bit state in a VGPR. The kernel is persistent: each
// workgroup stages the slot -> (symbol, f, slot - F) table in LDS once and its
// waves then walk over unit pairs.
//
// Per symbol group, going downwards (Sec. 2.2: the decoder consumes words in
// decreasing lane order before decoding a group):
//   read step   lanes with x < L take one 16-bit word each (Eq. 4). The lane's
//               word is the (count of reading lanes below it)-th of the words
//               the group consumes, a ballot plus mbcnt; words come from a
//               per-unit ring in LDS, so the dependent chain per group has two
//               LDS round trips and no global-memory latency;
//   decode step slot = x mod 2^n indexes the LDS table; x <- f (x >> n) + slot - F (Eq. 2);
//               the symbol is stored directly (64 consecutive bytes per wave).
//               For 13 <= n <= 16 the table has two levels (16-slot buckets,
//               then one entry per symbol), two LDS reads per symbol.
// Bitstream ring. Words are fetched in chunks of C = K*W words, the most a unit
// can consume in K groups (at most one word per symbol, since b >= n). A chunk
// is requested into registers at the start of a K-group super-step whenever
// fewer than 2C words remain resident, and written to the ring at its end, so
// the global-memory latency overlaps K groups of decoding. The ring holds
// 3C words plus a 64-word mirror of its first 64 slots, so a group's reads
// never wrap inside a wave.
// Synchronisation (Sec. 4.1.1). Lane j is switched on, with its recorded
// 16-bit state, at the read step of the group its recorded symbol belongs to,
// just before its first read. Groups above the unit's own range are decoded
// only to advance the states. The unit stores groups ghi .. glo (decoding and
// cross-boundary phases), so every output symbol is written by the unit that
// owns it. Once its states are exact, a run may keep decoding whole super-steps
// past glo (and the shorter run of a pair up to its partner's end); it then also
// stores the same symbols into the top groups of the run below (the run-on).
// Super-steps that contain synchronisation, the partial last group or the end
// of a unit run a predicated body; all others run the unpredicated one.
#include <algorithm>
#include <atomic>

#include "decode_core.hpp"

namespace recoil {

namespace {

using namespace dev;

// SS: units per wave. W = 32 runs two units per wave (one per half-wave), or,
// when the stream has no more units than the grid has waves, one unit per wave
// with the upper half-wave switched off: then twice as many waves decode.
template <int W, typename Sym, int K, int WAVES, int SS = 64 / W, int VAR = kPlain>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_num_sgpr(RECOIL_SGPR_BUDGET), amdgpu_waves_per_eu(8))) void decode_units(
    DecodeParams p) {
    using D = PairDecoder<W, Sym, K, SS, VAR>;
    using L = Lds<0, K, WAVES>;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *lut = smem + L::TABLE;
    const uint32_t base = lds_addr(smem);
    {
        const uint4 *src = static_cast<const uint4 *>(p.lut);
        const uint32_t chunks = p.lut_bytes / 16;
        for (uint32_t i = threadIdx.x; i < chunks; i += 64 * WAVES) reinterpret_cast<uint4 *>(lut)[i] = src[i];
    }
    __syncthreads();
    const uint32_t wave = uni(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (W * SS < 64 && lane >= (uint32_t)(W * SS)) return;   // lanes without a coder (no barrier follows)
    const uint32_t npairs = (p.runs + D::S - 1) / D::S;
    const uint32_t first = blockIdx.x * WAVES + wave, stride = gridDim.x * WAVES;
    D d(p, base + L::TABLE, base + L::PAD + wave * L::WAVE_LDS, lane);
    // Pairs are dealt out by position. The issue arbiter favours older waves,
    // which would leave the youngest waves holding the last pairs of the launch
    // alone (a shared work counter costs more: same-address atomics serialise).
    // Instead each wave's priority follows the part of its share still left.
    const uint32_t share = first < npairs ? (npairs - 1 - first) / stride + 1 : 0u;
    uint32_t left = share;
    for (uint32_t pair = first; pair < npairs; pair += stride) d.run(pair, --left, share);
}

template <typename Sym>
__global__ __launch_bounds__(256) void fill_symbol(Sym *out, uint64_t n, Sym v) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) out[i] = v;
}

template <int K, int WAVES>
size_t lds_bytes(uint32_t lut_bytes) {
    return Lds<0, K, WAVES>::TABLE + (size_t)lut_bytes;
}

template <int W, typename Sym, int K, int WAVES, int SS, int VAR>
int units_occupancy(uint32_t lut_bytes) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_units<W, Sym, K, WAVES, SS, VAR>, 64 * WAVES,
                                                     lds_bytes<K, WAVES>(lut_bytes)) != hipSuccess)
        return 0;
    return per_cu;
}

// Resident workgroups of the kernel with SS units per wave (0: does not fit).
template <int W, typename Sym, int K, int WAVES, int SS, int VAR>
uint32_t resident_blocks(const DecodeParams &p, const DecodeTuning &t) {
    int per_cu = units_occupancy<W, Sym, K, WAVES, SS, VAR>(p.lut_bytes);
    if (per_cu < 1) return 0;
    if (t.blocks_per_cu > 0) per_cu = std::min<int>(per_cu, (int)t.blocks_per_cu);
    return (uint32_t)(device_cus() * per_cu);
}

template <int W, typename Sym, int K, int WAVES, int SS, int VAR>
hipError_t launch_ss(const DecodeParams &p, const DecodeTuning &t, uint32_t resident, hipStream_t stream,
                     DecodeShape *shape) {
    DecodeParams q = p;
    q.run = t.units_per_run ? t.units_per_run : auto_units_per_run(p.units, (uint64_t)resident * WAVES * SS);
    q.run = std::min(q.run, std::max(p.units, 1u));
    if (p.partitioned) q.run = 1;   // independent sub-sequences cannot be decoded as one
    q.runs = (uint32_t)(((uint64_t)p.units + q.run - 1) / q.run);
    const uint32_t pairs = (q.runs + SS - 1) / SS;
    const uint32_t need = (pairs + WAVES - 1) / WAVES;
    const uint32_t blocks = std::max<uint32_t>(1u, std::min<uint32_t>(need, resident));
    if (shape) {
        *shape = DecodeShape{blocks, (uint32_t)WAVES, q.run, q.runs, (uint32_t)SS};
        return hipSuccess;
    }
    const size_t lds = lds_bytes<K, WAVES>(p.lut_bytes);
    hipLaunchKernelGGL((decode_units<W, Sym, K, WAVES, SS, VAR>), dim3(blocks), dim3(64 * WAVES), lds, stream, q);
    return hipGetLastError();
}

template <int W, typename Sym, int K, int WAVES, int VAR>
hipError_t launch_units(const DecodeParams &p, const DecodeTuning &t, hipStream_t stream, DecodeShape *shape) {
    if constexpr (W == 32) {
        // One unit per wave when every run then has a wave of its own: the
        // pair kernel would leave half of those waves idle.
        const uint32_t rs = resident_blocks<32, Sym, K, WAVES, 1, VAR>(p, t);
        const uint64_t slots = (uint64_t)rs * WAVES;
        const uint32_t k = t.units_per_run && !p.partitioned ? std::min(t.units_per_run, std::max(p.units, 1u)) : 1u;
        const uint64_t runs = ((uint64_t)p.units + k - 1) / k;
        if (rs > 0 && runs <= slots) return launch_ss<32, Sym, K, WAVES, 1, VAR>(p, t, rs, stream, shape);
    }
    const uint32_t resident = resident_blocks<W, Sym, K, WAVES, 64 / W, VAR>(p, t);
    if (resident == 0) return hipErrorInvalidConfiguration;
    return launch_ss<W, Sym, K, WAVES, 64 / W, VAR>(p, t, resident, stream, shape);
}

constexpr uint32_t kSimdsPerCu = 4;

template <int W, typename Sym, int VAR>
hipError_t launch_shape(const DecodeParams &p, const DecodeTuning &t, hipStream_t stream, DecodeShape *shape) {
    if (t.waves == 0) {
        // Automatic: 16 waves per workgroup; one when the launch has no more
        // wave-sized pieces of work than the chip has SIMDs, and 8 when 16-wave
        // workgroups would not reach every CU. A 16-wave grid of few pieces puts
        // four waves on each SIMD of a few CUs and leaves the rest idle, while
        // each wave's decode is one latency-bound chain that runs faster with
        // fewer waves beside it.
        DecodeTuning u = t;
        u.waves = 16;
        DecodeShape s{};
        const hipError_t e = launch_shape<W, Sym, VAR>(p, u, stream, &s);
        if (e != hipSuccess) return e;
        const uint64_t pieces = s.units_per_wave ? (s.runs + s.units_per_wave - 1) / s.units_per_wave : 0;
        const uint64_t cus = (uint64_t)device_cus();
        if (pieces <= kSimdsPerCu * cus) u.waves = 1;
        else if (pieces < 16 * cus) u.waves = 8;
        return launch_shape<W, Sym, VAR>(p, u, stream, shape);
    }
    if (t.chunk_groups == 4 && t.waves == 1) return launch_units<W, Sym, 4, 1, VAR>(p, t, stream, shape);
    if (t.chunk_groups == 4 && t.waves == 16) return launch_units<W, Sym, 4, 16, VAR>(p, t, stream, shape);
    if (t.chunk_groups == 4 && t.waves == 8) return launch_units<W, Sym, 4, 8, VAR>(p, t, stream, shape);
    if constexpr (VAR != kAdaptive) {   // adaptive tables take the LDS of 8-group rings: K = 4 only
        if (t.chunk_groups == 8 && t.waves == 1) return launch_units<W, Sym, 8, 1, VAR>(p, t, stream, shape);
        if (t.chunk_groups == 8 && t.waves == 8) return launch_units<W, Sym, 8, 8, VAR>(p, t, stream, shape);
        if (t.chunk_groups == 8 && t.waves == 16) return launch_units<W, Sym, 8, 16, VAR>(p, t, stream, shape);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int device_cus() {
    constexpr int kCached = 64;
    static std::atomic<int> cached[kCached];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (dev >= 0 && dev < kCached) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 1;
    if (dev >= 0 && dev < kCached) cached[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

hipError_t launch_decode(const DecodeParams &p, uint32_t lanes, uint32_t symbol_bytes, const DecodeTuning &t,
                         hipStream_t stream, DecodeShape *shape) {
    if (shape) *shape = DecodeShape{0, 0, 0, 0, 0};
    if (p.n_symbols == 0) return hipSuccess;
    if (p.single_symbol) {
        if (shape) return hipSuccess;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((p.n_symbols + 255) / 256, 65536);
        if (symbol_bytes == 1)
            hipLaunchKernelGGL(fill_symbol<uint8_t>, dim3(blocks), dim3(256), 0, stream,
                               static_cast<uint8_t *>(p.out), p.n_symbols, (uint8_t)p.fill_symbol);
        else
            hipLaunchKernelGGL(fill_symbol<uint16_t>, dim3(blocks), dim3(256), 0, stream,
                               static_cast<uint16_t *>(p.out), p.n_symbols, (uint16_t)p.fill_symbol);
        return hipGetLastError();
    }
    if (p.lut_bytes % 16 || p.lut_bytes > kMaxTableBytes) return hipErrorInvalidValue;
    if (p.quant_bits > 12) {
        // Wide tables (two-level, 13 <= n <= 16): plain decoding only.
        if (p.counts || p.tidx) return hipErrorInvalidValue;
        if (lanes == 32 && symbol_bytes == 1) return launch_shape<32, uint8_t, kWide>(p, t, stream, shape);
        if (lanes == 64 && symbol_bytes == 1) return launch_shape<64, uint8_t, kWide>(p, t, stream, shape);
        if (lanes == 32 && symbol_bytes == 2) return launch_shape<32, uint16_t, kWide>(p, t, stream, shape);
        if (lanes == 64 && symbol_bytes == 2) return launch_shape<64, uint16_t, kWide>(p, t, stream, shape);
        return hipErrorInvalidValue;
    }
    if (p.tidx) {
        // Adaptive coding: per-symbol tables, uint8 symbols only.
        if (p.counts || symbol_bytes != 1) return hipErrorInvalidValue;
        if (lanes == 32) return launch_shape<32, uint8_t, kAdaptive>(p, t, stream, shape);
        if (lanes == 64) return launch_shape<64, uint8_t, kAdaptive>(p, t, stream, shape);
        return hipErrorInvalidValue;
    }
    if (p.counts) {
        // Checking launches: the same kernels, also counting every symbol store.
        if (lanes == 32 && symbol_bytes == 1) return launch_shape<32, uint8_t, kCount>(p, t, stream, shape);
        if (lanes == 64 && symbol_bytes == 1) return launch_shape<64, uint8_t, kCount>(p, t, stream, shape);
        if (lanes == 32 && symbol_bytes == 2) return launch_shape<32, uint16_t, kCount>(p, t, stream, shape);
        if (lanes == 64 && symbol_bytes == 2) return launch_shape<64, uint16_t, kCount>(p, t, stream, shape);
        return hipErrorInvalidValue;
    }
    if (lanes == 32 && symbol_bytes == 1) return launch_shape<32, uint8_t, kPlain>(p, t, stream, shape);
    if (lanes == 64 && symbol_bytes == 1) return launch_shape<64, uint8_t, kPlain>(p, t, stream, shape);
    if (lanes == 32 && symbol_bytes == 2) return launch_shape<32, uint16_t, kPlain>(p, t, stream, shape);
    if (lanes == 64 && symbol_bytes == 2) return launch_shape<64, uint16_t, kPlain>(p, t, stream, shape);
    return hipErrorInvalidValue;
}

}  // namespace recoil
