// Device core of the Recoil decoder shared by the single-stream and batched kernels:
// decode tables, ring geometry and the per-unit-pair decoder (see decode.hip for
// the design notes).
#pragma once

#include <type_traits>

#include "decode.hpp"

namespace recoil {
namespace dev {

constexpr uint32_t kL = 1u << 16;

template <typename Sym>
struct Table;

template <>
struct Table<uint8_t> {
    using Entry = uint32_t;
    __device__ static inline uint32_t step(const Entry *lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const Entry e = lut[x & mask];
        const uint32_t f = (e >> 8) & 0xFFFu;
        const uint32_t off = e >> 20;
        x = __umul24(f, x >> n) + off;
        return e;           // low byte is the symbol
    }
};

template <>
struct Table<uint16_t> {
    using Entry = uint2;
    __device__ static inline uint32_t step(const Entry *lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const Entry e = lut[x & mask];
        const uint32_t f = e.x & 0xFFFFu;
        const uint32_t off = e.x >> 16;
        x = __umul24(f, x >> n) + off;
        return e.y;
    }
};

template <int W, typename Sym, int K, int WAVES>
struct Geo {
    static constexpr uint32_t S = 64 / W;                 // units per wave
    static constexpr uint32_t C = K * W;                  // chunk words
    static constexpr uint32_t R = 3 * C;                  // ring words
    static constexpr uint32_t RING = R + 64;              // ring words incl. mirror
    static constexpr uint32_t WAVE_LDS = S * RING * 2;    // bytes of rings per wave
    static constexpr uint32_t RINGS = WAVES * WAVE_LDS;   // bytes of rings per workgroup
    static constexpr uint32_t LANE_BYTES = 2 * K;         // chunk bytes per lane
    using Chunk = typename std::conditional<LANE_BYTES == 16, uint4, uint2>::type;
    static_assert(sizeof(Chunk) == LANE_BYTES, "chunk slice must be 8 or 16 bytes");
    static_assert(C >= 64, "mirror needs chunks of at least 64 words");
    static_assert(RINGS < 65536, "rings must leave the table at a 16-bit LDS offset");
};

__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <int W, typename Sym, int K, int WAVES>
struct PairDecoder {
    using G = Geo<W, Sym, K, WAVES>;
    using T = Table<Sym>;
    using Entry = typename T::Entry;
    using Chunk = typename G::Chunk;
    static constexpr uint32_t S = G::S, C = G::C, R = G::R, RING = G::RING;

    const DecodeParams &p;
    unsigned char *smem;
    const Entry *lut;
    uint32_t ring0;        // byte offset of this wave's rings in LDS
    uint32_t lane, j, upper;
    uint32_t n, mask;

    // Per unit of the pair (wave-uniform).
    uint32_t valid[S], last[S], top[S], ghi[S], steps[S], sync[S];
    int32_t nxt[S];        // words left below the cursor (first unread word is nxt - 1)
    uint32_t slotn[S];     // ring slot of word nxt (mod R)
    int32_t fq[S];         // lowest chunk held in the ring
    // Per lane.
    uint32_t x, rec, act;
    bool active;

    __device__ PairDecoder(const DecodeParams &p_, unsigned char *smem_, const Entry *lut_, uint32_t ring0_,
                           uint32_t lane_)
        : p(p_), smem(smem_), lut(lut_), ring0(ring0_), lane(lane_) {
        j = lane & (W - 1);
        upper = (W == 32) ? (lane >> 5) : 0u;
        n = p.quant_bits;
        mask = (1u << n) - 1u;
    }

    template <typename V>
    __device__ static inline V pick(const V (&a)[S], uint32_t h) {
        if constexpr (S == 1) return a[0];
        else return h ? a[1] : a[0];
    }

    __device__ inline uint32_t ring_byte(uint32_t h, uint32_t slot) const { return ring0 + 2u * (h * RING + slot); }

    __device__ inline const Chunk *chunk_src(int32_t q) const {
        return reinterpret_cast<const Chunk *>(p.words + (uint64_t)(uint32_t)q * C) + j;
    }

    // Write one chunk slice (this lane's part of chunk q) into the ring, and its mirror copy.
    __device__ inline void put_chunk(int32_t q, const Chunk &v) {
        const uint32_t slot = (uint32_t)(q % 3) * C + K * j;
        *reinterpret_cast<Chunk *>(smem + ring_byte(upper, slot)) = v;
        if (slot < 64) *reinterpret_cast<Chunk *>(smem + ring_byte(upper, R + slot)) = v;
    }

    __device__ bool begin(uint32_t pair) {
        const uint32_t u0 = pair * S;
        bool any = false;
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            const uint32_t u = u0 + h;
            valid[h] = u < p.units;
            last[h] = valid[h] && u + 1 == p.units;
            UnitMeta m = {0, 0, 0, 1};
            if (valid[h]) m = p.meta[u];
            nxt[h] = (int32_t)uni(m.next);
            top[h] = uni(m.top);
            ghi[h] = uni(m.ghi);
            const uint32_t glo = uni(m.glo);
            steps[h] = (valid[h] && top[h] + 1 > glo) ? top[h] + 1 - glo : 0u;
            if (last[h]) sync[h] = (p.n_symbols % W) ? 1u : 0u;
            else sync[h] = valid[h] ? top[h] - ghi[h] + 1 : 0u;
            any = any || steps[h] > 0;
        }
        const uint32_t my_valid = pick(valid, upper);
        const uint32_t my_last = pick(last, upper);
        rec = my_valid ? p.lanes[(uint64_t)(u0 + upper) * W + j] : 0u;
        x = my_last ? rec : 0u;
        active = my_last != 0;
        act = my_last ? 0u : (rec >> 16);
        // Initial ring fill: the chunk holding word nxt-1 and the two below it.
        int32_t q0[S];
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            q0[h] = nxt[h] > 0 ? (nxt[h] - 1) / (int32_t)C : -1;
            fq[h] = q0[h] >= 2 ? q0[h] - 2 : 0;
            slotn[h] = (uint32_t)nxt[h] % R;
        }
        const int32_t my_q0 = pick(q0, upper);
        Chunk c0{}, c1{}, c2{};
        if (my_q0 >= 0) c0 = *chunk_src(my_q0);
        if (my_q0 >= 1) c1 = *chunk_src(my_q0 - 1);
        if (my_q0 >= 2) c2 = *chunk_src(my_q0 - 2);
        if (my_q0 >= 0) put_chunk(my_q0, c0);
        if (my_q0 >= 1) put_chunk(my_q0 - 1, c1);
        if (my_q0 >= 2) put_chunk(my_q0 - 2, c2);
        return any;
    }

    // Read step for one group: ballot, consumed-word bookkeeping, per-lane ring address.
    __device__ inline void read_step(bool need) {
        const uint64_t bal = __ballot(need);
        const uint32_t bl = (uint32_t)bal, bh = (uint32_t)(bal >> 32);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(bh, __builtin_amdgcn_mbcnt_lo(bl, 0u));
        uint32_t addr;
        if constexpr (W == 64) {
            const uint32_t cnt = __popcll(bal);
            uint32_t bs = slotn[0] - cnt;
            if ((int32_t)bs < 0) bs += R;
            slotn[0] = bs;
            nxt[0] -= (int32_t)cnt;
            addr = (below << 1) + ring_byte(0, bs);
        } else {
            const uint32_t cA = __popc(bl), cB = __popc(bh);
            uint32_t bsA = slotn[0] - cA, bsB = slotn[1] - cB;
            if ((int32_t)bsA < 0) bsA += R;
            if ((int32_t)bsB < 0) bsB += R;
            slotn[0] = bsA;
            slotn[1] = bsB;
            nxt[0] -= (int32_t)cA;
            nxt[1] -= (int32_t)cB;
            // Upper lanes count the lower half's readers too: fold that into their offset.
            const uint32_t dW = (RING + bsB - cA) - bsA;
            addr = ((__umul24(upper, dW) + below) << 1) + ring_byte(0, bsA);
        }
        if (need) x = (x << 16) | *reinterpret_cast<const uint16_t *>(smem + addr);
    }

    __device__ inline void group_fast(unsigned char *outh, uint32_t lane_off) {
        read_step(x < kL);
        const uint32_t s = T::step(lut, x, n, mask);
        *reinterpret_cast<Sym *>(outh + lane_off) = (Sym)s;
    }

    __device__ inline void group_pred(uint32_t k) {
        const uint32_t my_steps = pick(steps, upper);
        const bool live = k < my_steps;
        if (live && !active && k == act) {
            active = true;
            x = rec & 0xFFFFu;
        }
        read_step(live && active && x < kL);
        const uint32_t h = pick(top, upper) - k;
        const uint64_t i = (uint64_t)h * W + j;
        if (live && active && i < p.n_symbols) {
            const uint32_t s = T::step(lut, x, n, mask);
            if (h <= pick(ghi, upper)) static_cast<Sym *>(p.out)[i] = (Sym)s;
        }
    }

    template <bool PRED>
    __device__ inline bool super_step(uint32_t k) {
        // Prefetch the next chunk of any unit that has fewer than 2C words resident.
        bool ld[S];
#pragma unroll
        for (uint32_t h = 0; h < S; ++h)
            ld[h] = steps[h] > k && fq[h] > 0 && nxt[h] - fq[h] * (int32_t)C < 2 * (int32_t)C;
        const bool my_ld = pick(ld, upper);
        const int32_t my_q = pick(fq, upper) - 1;
        Chunk pre{};
        if (my_ld) pre = *chunk_src(my_q);
        if constexpr (PRED) {
#pragma unroll
            for (uint32_t g = 0; g < K; ++g) group_pred(k + g);
        } else {
            // Unit A's group pointer is uniform; unit B's offset from it is per lane and fixed.
            unsigned char *outh = static_cast<unsigned char *>(p.out) + (uint64_t)(top[0] - k) * W * sizeof(Sym);
            uint32_t lane_off = j;
            if constexpr (S == 2) lane_off += upper * W * (top[1] - top[0]);
            lane_off *= sizeof(Sym);
#pragma unroll
            for (uint32_t g = 0; g < K; ++g) {
                group_fast(outh, lane_off);
                outh -= W * sizeof(Sym);
            }
        }
        if (my_ld) put_chunk(my_q, pre);
        bool ok = true;
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            if (ld[h]) fq[h] -= 1;
            if (valid[h] && nxt[h] < 0) ok = false;    // ran below the first word: corrupt split data
        }
        return ok;
    }

    __device__ void run(uint32_t pair) {
        if (!begin(pair)) return;
        uint32_t kmax = 0, kmin = 0xFFFFFFFFu, presync = 0;
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            kmax = max(kmax, steps[h]);
            kmin = min(kmin, steps[h]);
            presync = max(presync, sync[h]);
        }
        for (uint32_t k = 0; k < kmax; k += K) {
            const bool pred = k < presync || k + K > kmin;
            const bool ok = pred ? super_step<true>(k) : super_step<false>(k);
            if (!ok) {
                if (lane == 0) atomicOr(p.err, RECOIL_DEVERR_UNDERFLOW_BIT);
                return;
            }
        }
    }

    static constexpr uint32_t RECOIL_DEVERR_UNDERFLOW_BIT = 1u;
};


}  // namespace dev
}  // namespace recoil
