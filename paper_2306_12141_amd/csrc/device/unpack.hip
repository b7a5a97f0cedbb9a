// Split-point metadata unpacking on the device (Sec. 4.3). The two series have
// fixed-width entries, so split point k's entries sit at a computable bit
// position. The blocks have data-dependent widths, so each block's bit offset is
// handed in (recorded when the section is packed or checked on the host). One
// wave per output unit: lane j reads lane j's state and group difference, the
// wave reduces the differences to the unit's synchronisation group, and the
// unit's lowest group comes from the previous kept split point, which the same
// wave reads as well.
#include "unpack.hpp"

namespace recoil {
namespace {

constexpr uint32_t kWavesPerBlock = 4;

// `w` (1..32) bits at bit position `pos`, most significant bit first.
__device__ inline uint32_t bits_at(const uint8_t *p, uint64_t pos, uint32_t w) {
    const uint8_t *q = p + (pos >> 3);
    const uint64_t v = ((uint64_t)q[0] << 32) | ((uint64_t)q[1] << 24) | ((uint64_t)q[2] << 16) |
                       ((uint64_t)q[3] << 8) | (uint64_t)q[4];
    const uint32_t sh = 40u - (uint32_t)(pos & 7) - w;
    return (uint32_t)((v >> sh) & ((1ull << w) - 1));
}

// Entry k of a signed series whose width field starts at bit `at`.
__device__ inline int64_t series_entry(const uint8_t *p, uint64_t at, uint64_t k) {
    const uint32_t w = bits_at(p, at, 5) + 1;
    const uint64_t pos = at + 5 + k * (1 + w);
    const int64_t m = bits_at(p, pos + 1, w);
    return bits_at(p, pos, 1) ? -m : m;
}

__device__ inline uint32_t wave_max(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void unpack_units(UnpackParams p) {
    const uint32_t u = blockIdx.x * kWavesPerBlock + threadIdx.x / 64;
    const uint32_t j = threadIdx.x % 64;
    if (u >= p.units) return;                      // whole waves leave together
    const uint32_t W = p.lanes_per_unit;
    const bool lane = j < W;
    const uint64_t gtop = p.groups ? p.groups - 1 : 0;
    // The group series follows the offset series: 5 + (M-1)(1 + width) bits.
    const uint64_t x_at = p.splits > 1 ? 5 + (uint64_t)(p.splits - 1) * (2 + bits_at(p.bits, 0, 5)) : 0;

    // Split point k: its anchor group (clamped to the stream) and the group at
    // which all its lanes are switched on; lane j's state and difference on request.
    struct Split { uint32_t top, ghi; };
    auto split = [&](uint64_t k, uint32_t *state, uint32_t *gd) {
        const int64_t x = series_entry(p.bits, x_at, k);
        const uint32_t top = (uint32_t)min<int64_t>(max<int64_t>((int64_t)((k + 1) * p.eg) + x - 1, 0), (int64_t)gtop);
        const uint64_t bb = p.block_bit[k];
        const uint32_t wd = bits_at(p.bits, bb + 16ull * W, 4) + 1;
        const uint32_t d = lane ? bits_at(p.bits, bb + 16ull * W + 4 + (uint64_t)j * wd, wd) : 0u;
        if (state) *state = lane ? bits_at(p.bits, bb + 16ull * j, 16) : 0u;
        if (gd) *gd = d;
        return Split{top, top - min(wave_max(d), top)};
    };

    UnitMeta m;
    uint32_t word;
    if (u + 1 == p.units) {
        m.next = (uint32_t)p.words;
        m.top = (uint32_t)gtop;
        m.ghi = m.top;
        word = lane ? p.final_states[j] : 0u;
    } else {
        const uint64_t k = (uint64_t)(u + 1) * p.step - 1;
        const int64_t next = (int64_t)((k + 1) * p.eb) + series_entry(p.bits, 0, k);
        uint32_t state = 0, gd = 0;
        const Split s = split(k, &state, &gd);
        m.next = (uint32_t)min<int64_t>(max<int64_t>(next, 0), (int64_t)p.words);
        m.top = s.top;
        m.ghi = s.ghi;
        word = state | (gd << 16);
    }
    m.glo = u == 0 ? 0u : split((uint64_t)u * p.step - 1, nullptr, nullptr).ghi + 1;
    if (lane) p.lanes[(uint64_t)u * W + j] = word;
    if (j == 0) p.meta[u] = m;
}

}  // namespace

hipError_t launch_unpack(const UnpackParams &p, hipStream_t stream) {
    if (p.units == 0) return hipSuccess;
    const uint32_t blocks = (p.units + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(unpack_units, dim3(blocks), dim3(64 * kWavesPerBlock), 0, stream, p);
    return hipGetLastError();
}

}  // namespace recoil
