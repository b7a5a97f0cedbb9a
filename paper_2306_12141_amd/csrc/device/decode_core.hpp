// Device core of the Recoil decoder, shared by the single-stream and batched
// kernels (Lin et al., ICPP 2023, Sec. 4.1; Eq. 2 and Eq. 4).
//
// A decode unit is W interleaved rANS lanes; a 64-lane wavefront runs one unit
// (W = 64) or two (W = 32, one per half-wave). Coder j of a unit lives in wave
// lane W-1-j of its half, so that "reading lanes with a higher coder index",
// the words a lane must skip because the decoder consumes words in decreasing
// coder order (Sec. 2.2), are exactly the reading lanes below it in the wave:
// its offset is one mbcnt of the read ballot, independent of how many lanes
// read in total.
//
// Bitstream ring (per unit, in LDS). Words are fetched from HBM in chunks of
// C = K*W words, the most a unit can consume in a super-step of K groups (one
// word per symbol at most, since b >= n). A chunk is requested into registers
// at the start of a super-step whenever fewer than 2C words stay resident and is
// written to the ring at its end. The ring has 3C slots plus a C-word mirror of
// its top chunk placed below slot 0, so reads never wrap inside a super-step:
// word w lives at slot w mod 3C, and positions down to -C read the mirror.
//
// Per group the scalar unit only advances the LDS address of the unit's next
// word by twice the number of reading lanes (one s_bcnt1 and one s_lshl1_add
// per unit); the per-group store offsets are immediates of the unrolled
// super-step. The ring read is unconditional and selected with v_cndmask.
//
// Synchronisation (Sec. 4.1.1): lane j is switched on with its recorded 16-bit
// state at the read step of the group its recorded symbol belongs to, just
// before its first read; groups above the unit's range only advance states.
// The synchronisation lead-in runs a predicated body (a lean one when no unit
// of the pair is the stream's last), and so do a ragged last group and units
// that end near group 0 or word 0; all other super-steps run the unpredicated
// body. A run of consecutive units is decoded as one unit from its highest
// unit's split point (Sec. 3.3).
#pragma once

#include <type_traits>

#include "decode.hpp"

namespace recoil {
namespace dev {

constexpr uint32_t kL = 1u << 16;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kDevErrUnderflow = 1u;

// LDS is addressed with plain 32-bit LDS addresses (address space 3), so that
// uniform parts of an address stay in SGPRs and constants fold into the
// instructions' immediate offsets.
template <typename V>
__device__ inline V lds_ld(uint32_t a) {
    return *reinterpret_cast<const __attribute__((address_space(3))) V *>((size_t)a);
}
template <typename V>
__device__ inline void lds_st(uint32_t a, const V &v) {
    *reinterpret_cast<__attribute__((address_space(3))) V *>((size_t)a) = v;
}
__device__ inline uint32_t lds_addr(unsigned char *generic) {
    return (uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char *)generic;
}

template <typename Sym>
struct Table;

template <>
struct Table<uint8_t> {
    using Entry = uint32_t;   // symbol | f << 8 | (slot - F) << 20
    __device__ static inline uint32_t step(uint32_t lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const Entry e = lds_ld<Entry>(lut + ((x & mask) << 2));
        const uint32_t f = (e >> 8) & 0xFFFu;
        x = __umul24(f, x >> n) + (e >> 20);
        return e;             // the low byte is the symbol
    }
    // Adaptive coding: the symbol's own table t of the 2^n-entry tables laid end to end.
    __device__ static inline uint32_t step_t(uint32_t lut, uint32_t &x, uint32_t n, uint32_t mask, uint32_t t) {
        const Entry e = lds_ld<Entry>(lut + (((t << n) | (x & mask)) << 2));
        const uint32_t f = (e >> 8) & 0xFFFu;
        x = __umul24(f, x >> n) + (e >> 20);
        return e;
    }
};

template <>
struct Table<uint16_t> {
    using Entry = u32x2;      // .x = f | (slot - F) << 16, .y = symbol
    __device__ static inline uint32_t step(uint32_t lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const Entry e = lds_ld<Entry>(lut + ((x & mask) << 3));
        x = __umul24(e.x & 0xFFFFu, x >> n) + (e.x >> 16);
        return e.y;
    }
};

// Wide tables (13 <= n <= 16): the two-level layout of decode.hpp. The symbol's
// rank is the bucket's first rank plus the range starts between the bucket's first
// slot and this one (a popcount of the low p start bits, p = slot mod 16).
template <typename Sym>
struct WideTable {
    using Entry = u32x2;
    __device__ static inline uint32_t step(uint32_t lut, uint32_t &x, uint32_t n, uint32_t mask) {
        const uint32_t slot = x & mask;
        const uint32_t c = lds_ld<uint32_t>(lut + ((slot >> 4) << 2));
        const uint32_t r = (c >> 16) + __builtin_popcount(__builtin_amdgcn_ubfe(c, 0, slot & 15u));
        const Entry e = lds_ld<Entry>(lut + ((mask + 1u) >> 2) + (r << 3));
        x = __umul24(e.x, x >> n) + slot - (e.y >> 16);
        return e.y;
    }
};

template <int W, int K, int SS = 64 / W>
struct Geo {
    static constexpr uint32_t S = SS;                 // units per wave (W = 32: one per half-wave, or one)
    static constexpr uint32_t C = K * W;              // chunk words
    static constexpr uint32_t R = 3 * C;              // ring slots
    static constexpr uint32_t UNIT = 2 * (C + R);     // LDS bytes per unit: mirror + ring
    static constexpr uint32_t WAVE_LDS = S * UNIT;
    static constexpr uint32_t LANE_BYTES = 2 * K;     // chunk bytes per lane of a unit
    using Chunk = typename std::conditional<LANE_BYTES == 16, u32x4, u32x2>::type;
    static_assert(sizeof(Chunk) == LANE_BYTES, "chunk slice must be 8 or 16 bytes");
};

// LDS layout of a workgroup: [pad][rings of every wave][decode table]. The
// pad is a 16-byte slot the batched kernel uses to broadcast its work item.
template <int PADB, int K, int WAVES>
struct Lds {
    static constexpr uint32_t PAD = PADB;
    static constexpr uint32_t WAVE_LDS = Geo<32, K>::WAVE_LDS > Geo<64, K>::WAVE_LDS ? Geo<32, K>::WAVE_LDS
                                                                                     : Geo<64, K>::WAVE_LDS;
    static constexpr uint32_t TABLE = PAD + WAVES * WAVE_LDS;
};

__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// (x << 1) + y on the scalar unit in one instruction; the compiler emits a
// shift and an add for it.
__device__ inline uint32_t s_lshl1_add(uint32_t x, uint32_t y) {
    uint32_t r;
    asm("s_lshl1_add_u32 %0, %1, %2" : "=s"(r) : "s"(x), "s"(y) : "scc");
    return r;
}

// Wave issue priority 0..3 (larger values go first; the level is clamped).
__device__ inline void set_priority(uint32_t level) {
    if (level >= 3) __builtin_amdgcn_s_setprio(3);
    else if (level == 2) __builtin_amdgcn_s_setprio(2);
    else if (level == 1) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// A wave-uniform record read from global memory: every dword through
// readfirstlane, so its fields live in SGPRs rather than in VGPR copies.
template <typename T>
__device__ inline T uni_load(const T *src) {
    static_assert(sizeof(T) % 4 == 0, "record of whole dwords");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, src, sizeof(T));
#pragma unroll
    for (uint32_t i = 0; i < sizeof(T) / 4; ++i) w[i] = uni(w[i]);
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// Scalar registers per wave for the decode kernels. A SIMD held eight waves of
// a kernel using 62 of them but only seven at 76 (measured per-wave start
// times), and the decode loop needs every wave it can get to hide its LDS
// latency, so the kernels are compiled to this budget (the values that do not
// fit are kept in VGPR lanes and mostly reloaded outside the group loops).
#define RECOIL_SGPR_BUDGET 64

// Kernel variants: kCount also adds 1 to counts[i] for every store of symbol i (a
// checking launch); kAdaptive codes symbol i with decode table tidx[i] (adaptive
// coding, uint8 symbols); kWide reads the two-level table of 13 <= n <= 16.
constexpr int kPlain = 0, kCount = 1, kAdaptive = 2, kWide = 3;

template <int W, typename Sym, int K, int SS = 64 / W, int VAR = kPlain>
struct PairDecoder {
    using G = Geo<W, K, SS>;
    using T = typename std::conditional<VAR == kWide, WideTable<Sym>, Table<Sym>>::type;
    using Chunk = typename G::Chunk;
    static constexpr uint32_t S = G::S, C = G::C, R = G::R;
    static constexpr bool COUNT = VAR == kCount, ADAPT = VAR == kAdaptive;
    // Fast-body stores of byte symbols four groups at a time (see store_quad), for
    // 32-lane units: there a byte store writes only 32 bytes per unit, and one
    // dword store per four groups decoded W = 32 streams 13-16 % faster, while at
    // W = 64 the transpose's seven VALU per four groups cost more than the three
    // stores they save (1 % slower).
    static constexpr bool QUAD = W == 32 && sizeof(Sym) == 1 && K % 4 == 0;
    static_assert(!ADAPT || sizeof(Sym) == 1, "adaptive decoding reads the table index at the symbol's byte offset");

    const DecodeParams &p;
    uint32_t lut;          // LDS address of the decode table
    uint32_t ring0;        // LDS address of this wave's first unit
    uint32_t lane, col, upper, coder;
    uint32_t lane_ring;    // this lane's chunk-slice address in the top third of its unit's ring
    uint32_t n, mask;

    // Per unit of the pair (wave-uniform). Kept few: the register file holds
    // eight waves per SIMD only while a wave needs at most 64 scalar registers.
    uint32_t top0;         // unit 0's first group (the fast body's store base)
    uint32_t top_min;      // smallest first group of the pair's units
    uint32_t steps[S];     // groups the unit decodes
    uint32_t ua[S];        // LDS byte address of the unit's next word in its ring
    uint32_t presync;      // leading groups of the pair that need the predicated body
    bool sync_lean;        // no unit of the pair is the stream's last (ragged top group, 32-bit states)
    // Per lane, for the unit of the lane's half-wave: its ring bookkeeping lives in
    // vector registers, so one instruction keeps both units of a pair up to date and
    // the scalar registers hold only what the group loop needs.
    int32_t vres;          // words of the unit still in the ring: (next word + 1) - vfq * C
    int32_t vfq;           // lowest chunk held in the ring (the next fetch is vfq - 1)
    uint32_t vpo;          // byte offset from the top third of the third that chunk vfq - 1 goes to
    // Pairs (S == 2): the LDS byte address of the next word of the lane's unit, the
    // address at which it wraps, and a mask that confines a read ballot to the
    // lane's own half-wave.
    uint32_t vb, vlim, lowmask;
    // Adaptive coding: the table indices of the fast super-steps k and k + K (fetched
    // a super-step ahead; tready: tcur already holds super-step k's). A predicated or
    // synchronisation super-step fetches its own into tcur at its start (those run
    // outside the fast loops, so the registers are free then).
    uint32_t tcur[K], tn1[K];
    uint32_t tready = 0;
    uint32_t x, rec, act, lim;
    uint32_t my_top, my_ghi, my_steps, lane_off;
    uint32_t quad_off;     // QUAD: this lane's dword offset from the fast body's group pointer, plus 3W
    bool active;

    __device__ PairDecoder(const DecodeParams &p_, uint32_t lut_, uint32_t ring0_, uint32_t lane_)
        : p(p_), lut(lut_), ring0(ring0_), lane(lane_) {
        col = lane & (W - 1);
        upper = (S == 2) ? (lane >> 5) : 0u;
        coder = W - 1 - col;
        n = p.quant_bits;
        mask = (1u << n) - 1u;
        lane_ring = lane_ring_addr();
    }

    // LDS byte address of ring position s (s in [-C, R)) of unit h. The ring is
    // stored in descending order (slot R-1 lowest, the mirror of slots 2C..3C-1
    // above slot 0), so consecutive reads of a group go upwards in LDS.
    __device__ inline uint32_t ring_addr(uint32_t h, int32_t s) const {
        return ring0 + h * G::UNIT + 2u * (uint32_t)((int32_t)R - 1 - s);
    }

    // Byte offset, from the top third, of the third holding chunk q.
    __device__ static inline uint32_t third_off(int32_t q) { return 2u * C * (uint32_t)(2 - q % 3); }

    // This lane's slice of chunk q (uniform q): a scalar base plus a fixed lane offset.
    __device__ inline Chunk fetch(int32_t q) const {
        const unsigned char *base = reinterpret_cast<const unsigned char *>(p.words) + (uint64_t)(uint32_t)q * (2 * C);
        return *reinterpret_cast<const Chunk *>(base + col * (uint32_t)sizeof(Chunk));
    }

    // This lane's slice (K words, ascending) of a chunk into the ring third at
    // byte offset off from the top third, words reversed; the top third is also
    // written to the mirror below slot 0.
    __device__ inline void put_chunk(uint32_t off, const Chunk &v) {
        Chunk r16;
        if constexpr (K == 4) {
            r16.x = __builtin_amdgcn_alignbit(v.y, v.y, 16);
            r16.y = __builtin_amdgcn_alignbit(v.x, v.x, 16);
        } else {
            r16.x = __builtin_amdgcn_alignbit(v.w, v.w, 16);
            r16.y = __builtin_amdgcn_alignbit(v.z, v.z, 16);
            r16.z = __builtin_amdgcn_alignbit(v.y, v.y, 16);
            r16.w = __builtin_amdgcn_alignbit(v.x, v.x, 16);
        }
        lds_st<Chunk>(lane_ring + off, r16);
        if (off == 0) lds_st<Chunk>(lane_ring + 6 * C, r16);
    }

    // Lane slice address for chunks in the top third of the ring.
    __device__ inline uint32_t lane_ring_addr() const { return ring_addr(upper, 2 * (int32_t)C + (int32_t)(K * col + K - 1)); }

    // A run of consecutive units decodes as one unit: it starts from its
    // highest unit's split point (records, first word, first group, completion
    // point) and ends at its lowest unit's last group; the split points in
    // between are not used (Sec. 3.3).
    __device__ bool begin(uint32_t pair) {
        const uint32_t r0 = pair * S;
        bool any = false;
        bool has_last = false;
        uint32_t sync_max = 0;
        int32_t cur[S];
        uint32_t top[S], ghi[S];
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            const uint32_t r = r0 + h;
            const bool valid = r < p.runs;
            const uint32_t lo = r * p.run;
            const uint32_t hi = valid ? min(lo + p.run, p.units) - 1u : 0u;
            const bool last = valid && hi + 1 == p.units;
            const bool full = last || (valid && p.partitioned);   // starts from 32-bit final states
            UnitMeta m = {0, 0, 0, 1};
            if (valid) {
                m = p.meta[hi];
                m.glo = p.meta[lo].glo;
            }
            cur[h] = (int32_t)uni(m.next);
            top[h] = uni(m.top);
            ghi[h] = uni(m.ghi);
            const uint32_t glo = uni(m.glo);
            steps[h] = (valid && top[h] + 1 > glo) ? top[h] + 1 - glo : 0u;
            uint32_t sync = valid ? top[h] - ghi[h] + 1 : 0u;
            if (full) sync = (last && (p.n_symbols % W)) ? 1u : 0u;   // only the stream's last group is ragged
            has_last = has_last || full;
            sync_max = max(sync_max, sync);
            any = any || steps[h] > 0;
        }
        presync = sync_max;
        sync_lean = !has_last;
        top0 = top[0];
        top_min = S == 2 ? min(top[0], top[S - 1]) : top[0];
        my_top = S == 2 && upper ? top[S - 1] : top[0];
        my_ghi = S == 2 && upper ? ghi[S - 1] : ghi[0];
        my_steps = S == 2 && upper ? steps[S - 1] : steps[0];
        // Fast-body store offset of this lane from unit 0's group pointer.
        lane_off = (coder + (S == 2 ? upper * W * (my_top - top0) : 0u)) * (uint32_t)sizeof(Sym);
        // Lane 4a + b of a quad writes group b of a block of four, at the column of
        // the quad's highest lane (its lowest coder): 3 - b columns below its own.
        quad_off = lane_off - 3u + (lane & 3u) + (3u - (lane & 3u)) * W;
        const uint32_t mine = r0 + upper;
        const bool my_valid = mine < p.runs;
        const uint32_t my_hi = my_valid ? min(mine * p.run + p.run, p.units) - 1u : 0u;
        const bool my_full = my_valid && (my_hi + 1 == p.units || p.partitioned);
        rec = my_valid ? p.lanes[(uint64_t)my_hi * W + coder] : 0u;
        x = my_full ? rec : 0u;
        active = my_full;
        act = my_full ? 0u : (rec >> 16);
        // Initial fill: the chunk holding word cur-1 and the two below it.
        int32_t q0[S], fq[S], res[S];
        uint32_t po[S];
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            q0[h] = cur[h] > 0 ? (cur[h] - 1) / (int32_t)C : -1;
            fq[h] = q0[h] >= 2 ? q0[h] - 2 : 0;
            res[h] = cur[h] - fq[h] * (int32_t)C;
            ua[h] = uni(ring_addr(h, cur[h] > 0 ? (cur[h] - 1) % (int32_t)R : 0));
            po[h] = third_off(fq[h] + 2);      // chunk fq - 1 shares a third with fq + 2
        }
        const bool hi = S == 2 && upper;
        vfq = hi ? fq[S - 1] : fq[0];
        vres = hi ? res[S - 1] : res[0];
        vpo = hi ? po[S - 1] : po[0];
        if constexpr (S == 2) {
            vb = hi ? ua[S - 1] : ua[0];
            vlim = ring_addr(upper, -1);
            lowmask = upper ? 0u : 0xFFFFFFFFu;
        }
#pragma unroll
        for (uint32_t h = 0; h < S; ++h)
            for (int32_t q = q0[h]; q >= 0 && q > q0[h] - 3; --q)
                if (S == 1 || upper == h) put_chunk(third_off(q), fetch(q));
        return any;
    }

    // One group's read step. need is this lane's "x < L" (and live). For one unit
    // per wave, a is the unit's scalar LDS address of its next word; for a pair, e
    // is the lane's own unit's address (a vector register), so that the address
    // chain of a group (ballot, count, address, LDS read) has no scalar step.
    template <uint32_t G_IDX>
    __device__ inline void read_step(bool need, uint32_t &a, uint32_t &e) {
        const uint64_t bal = __ballot(need);
        const uint32_t bl = (uint32_t)bal, bh = (uint32_t)(bal >> 32);
        uint32_t addr;
        if constexpr (S == 1) {
            const uint32_t m = __builtin_amdgcn_mbcnt_hi(bh, __builtin_amdgcn_mbcnt_lo(bl, 0u));
            // The lane's word is m words above the unit's top word (descending ring);
            // a stays an opaque SGPR byte address so the address is one v_lshl_add.
            asm volatile("" : "+s"(a));
            addr = (m << 1) + a;
            a = s_lshl1_add((uint32_t)__builtin_popcountll(bal), a);
        } else {
            // Readers below the lane in its own half-wave: the lower half's ballot is
            // masked off for upper lanes before the count (one v_and with the scalar
            // ballot; the opaque mask keeps the compiler from turning it into selects).
            asm volatile("" : "+v"(lowmask));
            const uint32_t m = __builtin_amdgcn_mbcnt_hi(bh, __builtin_amdgcn_mbcnt_lo(bl & lowmask, 0u));
            addr = (m << 1) + e;
            // Each unit's address advances by twice its own readers, off the address
            // chain of this group: e += 2 pl + upper * 2 (ph - pl). (A VALU instruction
            // reads at most one scalar operand, so the two counts cannot be selected
            // per lane in one instruction.)
            const int32_t pl = __builtin_popcount(bl), ph = __builtin_popcount(bh);
            const int32_t dd = 2 * (ph - pl);
            uint32_t t;
            asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(t) : "v"(upper), "s"(dd), "v"(e));
            asm("v_lshl_add_u32 %0, %1, 1, %2" : "=v"(e) : "s"(pl), "v"(t));
        }
        uint32_t w = lds_ld<uint16_t>(addr);
        // Keep the read unconditional: lanes that do not need it read an in-ring word and drop it.
        asm volatile("" : "+v"(w));
        x = need ? ((x << 16) | w) : x;
    }

    // This lane's table indices of the K groups from group top0 - k down (the bytes
    // at its output offsets; only for groups inside the stream).
    __device__ inline void load_tidx(uint32_t k, uint32_t (&dst)[K]) const {
        const uint8_t *b = p.tidx + (uint64_t)(top0 - k) * W + lane_off;
#pragma unroll
        for (uint32_t g = 0; g < K; ++g) dst[g] = *(b - (int64_t)(g * W));
    }

    // The same for KK groups of a predicated or synchronisation super-step, where a
    // lane's group may lie outside its unit or the stream: those lanes load nothing.
    template <uint32_t KK>
    __device__ inline void load_tidx_checked(uint32_t k) {
#pragma unroll
        for (uint32_t g = 0; g < KK; ++g) {
            const uint32_t kk = k + g;
            const uint64_t i = (uint64_t)(my_top - kk) * W + coder;
            tcur[g] = (kk <= my_top && i < p.n_symbols) ? (uint32_t)p.tidx[i] : 0u;
        }
    }

    // Byte symbols of groups G0 .. G0 + 3 (the low bytes of v[0..3]) written as one
    // dword per lane: the four lanes of a quad hold four adjacent coders, so a 4 x 4
    // byte transpose across the quad (two DPP swaps, each followed by a byte
    // permute) leaves in lane 4a + b the four symbols of group G0 + b for coders
    // W-4-4a .. W-1-4a, in address order. One store per four groups replaces four
    // byte stores; the bytes written are the same.
    template <uint32_t G0>
    __device__ inline void store_quad(unsigned char *outh, const uint32_t (&v)[4]) const {
        const uint32_t b = lane & 3u;
        // d: byte j = this lane's symbol of group G0 + j.
        const uint32_t d = __builtin_amdgcn_perm(__builtin_amdgcn_perm(v[3], v[2], 0x00000400u),
                                                 __builtin_amdgcn_perm(v[1], v[0], 0x00000400u), 0x05040100u);
        // Swap 16-bit halves with lane b ^ 2: lanes 0, 1 keep groups 0-1, lanes 2, 3 groups 2-3.
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0x4E, 0xF, 0xF, false);
        const uint32_t h = __builtin_amdgcn_perm(p2, d, (b & 2u) ? 0x03020706u : 0x05040100u);
        // Swap bytes with lane b ^ 1 and order the coders upwards in address.
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)h, 0xB1, 0xF, 0xF, false);
        const uint32_t t = __builtin_amdgcn_perm(p1, h, (b & 1u) ? 0x05010703u : 0x00040206u);
        unsigned char *dst = outh + quad_off - (G0 + 3) * W;
        *reinterpret_cast<uint32_t *>(dst) = t;
        if constexpr (COUNT) {
            const uint64_t i = (uint64_t)(dst - static_cast<unsigned char *>(p.out));
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) count_store(i + j);
        }
    }

    template <uint32_t G_IDX>
    __device__ inline void group_fast(uint32_t &a, uint32_t &e, unsigned char *outh, uint32_t (&held)[4]) {
        read_step<G_IDX>(x < kL, a, e);
        uint32_t s;
        if constexpr (ADAPT) s = T::step_t(lut, x, n, mask, tcur[G_IDX]);
        else s = T::step(lut, x, n, mask);
        if constexpr (QUAD) {
            held[G_IDX & 3u] = s;
            if constexpr ((G_IDX & 3u) == 3u) store_quad<G_IDX - 3u>(outh, held);
        } else {
            unsigned char *dst = outh + lane_off - G_IDX * W * sizeof(Sym);
            *reinterpret_cast<Sym *>(dst) = (Sym)s;
            if constexpr (COUNT) count_store((uint64_t)(dst - static_cast<unsigned char *>(p.out)) / sizeof(Sym));
        }
    }

    __device__ inline void count_store(uint64_t i) const { atomicAdd(p.counts + i, 1u); }

    template <uint32_t G_IDX>
    __device__ inline void group_pred(uint32_t k, uint32_t &a, uint32_t &e) {
        const bool live = k < my_steps;
        if (live && !active && k == act) {
            active = true;
            x = rec & 0xFFFFu;
        }
        read_step<G_IDX>(live && active && x < kL, a, e);
        const uint32_t h = my_top - k;
        const uint64_t i = (uint64_t)h * W + coder;
        if (live && active && i < p.n_symbols) {
            uint32_t s;
            if constexpr (ADAPT) s = T::step_t(lut, x, n, mask, tcur[G_IDX]);
            else s = T::step(lut, x, n, mask);
            if (h <= my_ghi) {
                static_cast<Sym *>(p.out)[i] = (Sym)s;
                if constexpr (COUNT) count_store(i);
            }
        }
    }

    // Synchronisation group of a pair whose units are all within their own
    // groups and below the stream's last group: only the switching-on of lanes
    // and the stores of groups above a unit's completion point are predicated.
    // Lanes not yet on decode garbage that is dropped when they switch on.
    // A lane reads while x < lim, and lim turns from 0 to L when the lane is
    // switched on, so the read predicate stays a single compare.
    template <uint32_t G_IDX>
    __device__ inline void group_sync(uint32_t k, uint32_t &a, uint32_t &e) {
        const bool on = k == act;
        x = on ? (rec & 0xFFFFu) : x;
        lim = on ? kL : lim;
        read_step<G_IDX>(x < lim, a, e);
        uint32_t lb = lut;
        asm volatile("" : "+s"(lb));   // the table base as a scalar operand of the address
        const uint32_t h = my_top - k;
        uint32_t s;
        if constexpr (ADAPT) s = T::step_t(lb, x, n, mask, tcur[G_IDX]);
        else s = T::step(lb, x, n, mask);
        if (h <= my_ghi) {
            static_cast<Sym *>(p.out)[(uint64_t)h * W + coder] = (Sym)s;
            if constexpr (COUNT) count_store((uint64_t)h * W + coder);
        }
    }

    // Eighths of the share below which priority level L (1..3) ends.
    __device__ static inline uint32_t prio_cut(uint32_t L) { return L == 3 ? 4u : L == 2 ? 2u : 1u; }

    // Bodies of a super-step: unpredicated, synchronisation, fully predicated.
    static constexpr int kFast = 0, kSync = 1, kPred = 2;

    template <int MODE, uint32_t... G_IDX>
    __device__ inline void groups(std::integer_sequence<uint32_t, G_IDX...>, uint32_t k, uint32_t &a, uint32_t &e) {
        if constexpr (MODE == kPred) {
            (group_pred<G_IDX>(k + G_IDX, a, e), ...);
        } else if constexpr (MODE == kSync) {
            (group_sync<G_IDX>(k + G_IDX, a, e), ...);
        } else {
            unsigned char *outh = static_cast<unsigned char *>(p.out) + (uint64_t)(top0 - k) * W * sizeof(Sym);
            uint32_t held[4];
            (group_fast<G_IDX>(a, e, outh, held), ...);
        }
    }

    // K groups. At the start, every unit with fewer than 2C words resident
    // requests its next chunk into registers; the chunk is written to the ring
    // after the K groups, so the load overlaps them. (Every step consumes at
    // most C words, so a unit keeps at least C words resident, and reads stay
    // within the ring plus its mirror.) Returns false if a unit read past its
    // first word (corrupt split data).
    // fend: fast super-steps of the current loop are those at k' with k' + K <= fend.
    template <int MODE, uint32_t KK = K>
    __device__ inline bool super_step(uint32_t k, uint32_t fend = 0) {
        if constexpr (ADAPT && MODE == kFast) {
            // Table indices: this super-step's unless fetched ahead, and the next
            // one's when it is also fast (its groups are then inside the stream).
            if (!tready) load_tidx(k, tcur);
            if (k + 2 * K <= fend) load_tidx(k + K, tn1);
        } else if constexpr (ADAPT) {
            load_tidx_checked<KK>(k);
        }
        // Per lane: does this lane's unit fetch? (Uniform within each half-wave.)
        const bool need = (MODE != kPred || my_steps > k) && vfq > 0 && vres < 2 * (int32_t)C;
        uint32_t a = ua[0], e = S == 2 ? vb : 0u;
        if (__ballot(need)) {
            // One load for the whole wave, each unit's lanes addressing their own
            // chunk by a 32-bit byte offset from the scalar bitstream base (lanes of
            // a unit that does not fetch load an in-range chunk and drop it). The
            // registers stay untouched until the K groups are done; the empty asm
            // keeps the scheduler from hoisting the chunk's use (and its wait on
            // the load) into the groups.
            const uint32_t off = (uint32_t)max(vfq - 1, 0) * (2 * C);
            Chunk pre = *reinterpret_cast<const Chunk *>(reinterpret_cast<const unsigned char *>(p.words) +
                                                         (off + col * (uint32_t)sizeof(Chunk)));
            groups<MODE>(std::make_integer_sequence<uint32_t, KK>{}, k, a, e);
            asm volatile("" : "+v"(pre));
            if (need) {
                put_chunk(vpo, pre);
                vfq -= 1;
                vres += (int32_t)C;
                vpo = vpo == 4 * C ? 0u : vpo + 2 * C;
            }
        } else {
            groups<MODE>(std::make_integer_sequence<uint32_t, KK>{}, k, a, e);
        }
        // Words the lane's unit consumed, from its address advance; an address that
        // moved into the mirror (below slot 0) wraps to the ring's top.
        if constexpr (S == 1) {
            vres -= (int32_t)((a - ua[0]) >> 1);
            ua[0] = a >= ring_addr(0, -1) ? a - 2 * R : a;
        } else {
            vres -= (int32_t)((e - vb) >> 1);
            vb = e >= vlim ? e - 2 * R : e;
        }
        if constexpr (ADAPT && MODE == kFast) {
#pragma unroll
            for (uint32_t g = 0; g < K; ++g) tcur[g] = tn1[g];
            tready = k + 2 * K <= fend ? 1u : 0u;
        }
        return __ballot(vres < 0) == 0;   // read below the first word: corrupt split data
    }

    // Decodes one pair. left: pairs of the wave's share after this one.
    // The wave's issue priority follows the part of its share still to be
    // decoded (counted in groups with every pair as long as this one, updated
    // every super-step): 3 above one half, 2 above a quarter, 1 above an eighth,
    // else 0. The issue arbiter favours older waves; waves that fall behind are
    // given precedence so that all end together, and the last level, in which
    // the oldest wave goes first again, is kept short.
    __device__ void run(uint32_t pair, uint32_t left, uint32_t share) {
        if (!begin(pair)) return;
        uint32_t kmax = 0, kmin = 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t h = 0; h < S; ++h) {
            kmax = max(kmax, steps[h]);
            kmin = min(kmin, steps[h]);
        }
        // With rem = (left + 1) kmax - k and q = share kmax, level L > 0 holds while
        // 8 rem >= cut(L) q, i.e. until 8 k exceeds thr = 8 (left + 1) kmax - cut(L) q.
        const uint32_t q = share * kmax;
        const uint32_t r8 = 8 * (left + 1);
        uint32_t level = r8 > 4 * share ? 3u : r8 > 2 * share ? 2u : r8 > share ? 1u : 0u;
        uint32_t thr = level ? r8 * kmax - prio_cut(level) * q : 0xFFFFFFFFu;
        set_priority(level);
        // Synchronisation runs predicated, in half super-steps so that little
        // of the pair does.
        bool ok = true;
        uint32_t k = 0;
        // The lean body needs every unit within its own groups for the whole
        // lead-in; it does not track which lanes are on, so afterwards (when all
        // are) the flag is set for the predicated body of the end.
        const uint32_t lead = (presync + K / 2 - 1) / (K / 2) * (K / 2);
        if (sync_lean && lead <= kmin) {
            lim = 0;
            for (; ok && k < presync; k += K / 2) ok = super_step<kSync, K / 2>(k);
            active = true;
        } else {
            for (; ok && k < kmax && k < presync; k += K / 2) ok = super_step<kPred, K / 2>(k);
        }
        // From here every state of every unit is exact, so a unit that has
        // decoded its own groups may run on into the groups below: it stores
        // there the symbols the unit below stores too, and reads that unit's
        // words. The rest of the pair then runs unpredicated in whole super-steps,
        // provided every unit is still within its own groups here (a unit that
        // ended during synchronisation stopped advancing) and running on reaches
        // neither below group 0 nor below word 0 (the first units of the stream);
        // otherwise the end runs predicated.
        const uint32_t kend = k < kmax ? k + (kmax - k + K - 1) / K * K : k;
        // Independent sub-sequences (Sec. 2.3) never run on: the states do not carry
        // over into the sub-sequence below.
        bool run_on = !p.partitioned && k <= kmin && top_min + 1 >= kend;
        run_on = run_on && __ballot(vres + vfq * (int32_t)C < (int32_t)((kend - k) * W)) == 0;
        tready = 0;
        if (run_on) {
            for (; ok && k < kmax; k += K) {
                if (8 * k > thr) {
                    --level;
                    thr = level ? thr + (prio_cut(level + 1) - prio_cut(level)) * q : 0xFFFFFFFFu;
                    set_priority(level);
                }
                ok = super_step<kFast>(k, kend);
            }
        } else {
            for (; ok && k + K <= kmin; k += K) {
                if (8 * k > thr) {
                    --level;
                    thr = level ? thr + (prio_cut(level + 1) - prio_cut(level)) * q : 0xFFFFFFFFu;
                    set_priority(level);
                }
                ok = super_step<kFast>(k, kmin);
            }
            for (; ok && k < kmax; k += K) ok = super_step<kPred>(k);
        }
        if (!ok && lane == 0) atomicOr(p.err, kDevErrUnderflow);
    }
};

}  // namespace dev
}  // namespace recoil
