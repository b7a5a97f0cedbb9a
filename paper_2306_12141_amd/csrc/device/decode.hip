// Recoil split decoding on gfx950 (Lin et al., ICPP 2023, Sec. 4.1).
//
// Mapping: a decode unit is W interleaved rANS lanes; a 64-lane wavefront runs
// one unit (W = 64) or two (W = 32, one per half-wave). Lane j of a unit holds
// coder j's state in a VGPR. Per symbol group, going downwards:
//   read step   lanes whose state fell below L read one 16-bit word each, in
//               decreasing lane order (Sec. 2.2, Eq. 4); the per-lane offset is
//               the count of reading lanes above it in the unit, taken from a
//               ballot and a masked bit count;
//   decode step slot = x mod 2^n indexes the decode table in LDS, giving the
//               symbol, f and slot - F; x <- f (x >> n) + slot - F (Eq. 2).
// Synchronisation (Sec. 4.1.1): lane j is switched on, with its recorded 16-bit
// state, at the read step of the group its recorded symbol belongs to, i.e.
// just before its first read; symbols of groups above the unit's own range are
// decoded only to advance the states and are not stored. The unit stores
// groups ghi .. glo (its decoding and cross-boundary phases), so every output
// symbol is written by exactly one unit.
#include "decode.hpp"

namespace recoil {

namespace {

constexpr uint32_t kL = 1u << 16;
constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kBlock = kWaves * 64;

template <typename Sym>
struct Table;

template <>
struct Table<uint8_t> {
    using Entry = uint32_t;
    __device__ static inline uint32_t step(const Entry *lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const Entry e = lut[x & mask];
        const uint32_t f = (e >> 8) & 0xFFFu;
        const uint32_t off = e >> 20;
        x = f * (x >> n) + off;
        return e & 0xFFu;
    }
};

template <>
struct Table<uint16_t> {
    using Entry = uint2;
    __device__ static inline uint32_t step(const Entry *lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const Entry e = lut[x & mask];
        const uint32_t f = e.x & 0xFFFFu;
        const uint32_t off = e.x >> 16;
        x = f * (x >> n) + off;
        return e.y;
    }
};

template <int W, typename Sym>
__global__ __launch_bounds__(kBlock) void decode_units(DecodeParams p) {
    using T = Table<Sym>;
    using Entry = typename T::Entry;
    extern __shared__ __align__(16) unsigned char smem[];
    Entry *lut = reinterpret_cast<Entry *>(smem);
    const uint32_t n = p.quant_bits;
    const uint32_t mask = (1u << n) - 1u;
    {
        const Entry *src = static_cast<const Entry *>(p.lut);
        for (uint32_t i = threadIdx.x; i <= mask; i += kBlock) lut[i] = src[i];
    }
    __syncthreads();

    constexpr uint32_t S = 64 / W;   // units per wave
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t j = lane % W;
    const uint32_t unit = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * S + lane / W;
    const bool valid = unit < p.units;
    UnitMeta m = {0, 0, 0, 1};
    uint32_t rec = 0;
    if (valid) {
        m = p.meta[unit];
        rec = p.lanes[(uint64_t)unit * W + j];
    }
    const bool is_last = valid && unit + 1 == p.units;
    uint32_t x = is_last ? rec : 0u;
    bool active = is_last;
    const uint32_t act = is_last ? 0u : (rec >> 16);
    uint32_t steps = (valid && m.top + 1 > m.glo) ? m.top + 1 - m.glo : 0u;
    uint32_t next = m.next;
    Sym *out = static_cast<Sym *>(p.out);

    for (uint32_t k = 0;; ++k) {
        bool live = k < steps;
        if (!__any(live)) break;
        // Read step before group h (Sec. 4.1.1: activation happens right before a lane's first read).
        if (live && !active && k == act) {
            active = true;
            x = rec & 0xFFFFu;
        }
        const bool need = live && active && x < kL;
        const uint64_t ballot = __ballot(need);
        uint32_t cnt, below;
        if (W == 64) {
            cnt = (uint32_t)__popcll(ballot);
            below = (uint32_t)__popcll(ballot & ((1ull << lane) - 1ull));
        } else {
            const uint32_t hm = (uint32_t)(ballot >> (lane & 32u));
            cnt = (uint32_t)__popc(hm);
            below = (uint32_t)__popc(hm & ((1u << j) - 1u));
        }
        if (live && cnt > next) {
            // Corrupt metadata: the unit would read below the start of the bitstream.
            if (j == 0) atomicOr(p.err, 1u);
            steps = k;
            continue;
        }
        if (need) x = (x << 16) | p.words[next - cnt + below];
        next -= live ? cnt : 0u;
        // Decode group h (Eq. 2).
        const uint32_t h = m.top - k;
        const uint64_t i = (uint64_t)h * W + j;
        if (live && active && i < p.n_symbols) {
            const uint32_t s = T::step(lut, x, n, mask);
            if (h <= m.ghi) out[i] = (Sym)s;
        }
    }
}

template <typename Sym>
__global__ __launch_bounds__(256) void fill_symbol(Sym *out, uint64_t n, Sym v) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) out[i] = v;
}

template <int W, typename Sym>
hipError_t launch_units(const DecodeParams &p, hipStream_t stream) {
    const uint32_t per_block = kWaves * (64 / W);
    const uint32_t blocks = (p.units + per_block - 1) / per_block;
    const size_t lds = (size_t)sizeof(typename Table<Sym>::Entry) << p.quant_bits;
    hipLaunchKernelGGL((decode_units<W, Sym>), dim3(blocks), dim3(kBlock), lds, stream, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_decode(const DecodeParams &p, uint32_t lanes, uint32_t symbol_bytes, hipStream_t stream) {
    if (p.n_symbols == 0) return hipSuccess;
    if (p.single_symbol) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((p.n_symbols + 255) / 256, 65536);
        if (symbol_bytes == 1)
            hipLaunchKernelGGL(fill_symbol<uint8_t>, dim3(blocks), dim3(256), 0, stream,
                               static_cast<uint8_t *>(p.out), p.n_symbols, (uint8_t)p.fill_symbol);
        else
            hipLaunchKernelGGL(fill_symbol<uint16_t>, dim3(blocks), dim3(256), 0, stream,
                               static_cast<uint16_t *>(p.out), p.n_symbols, (uint16_t)p.fill_symbol);
        return hipGetLastError();
    }
    if (lanes == 32 && symbol_bytes == 1) return launch_units<32, uint8_t>(p, stream);
    if (lanes == 64 && symbol_bytes == 1) return launch_units<64, uint8_t>(p, stream);
    if (lanes == 32 && symbol_bytes == 2) return launch_units<32, uint16_t>(p, stream);
    if (lanes == 64 && symbol_bytes == 2) return launch_units<64, uint16_t>(p, stream);
    return hipErrorInvalidValue;
}

}  // namespace recoil
