// GPU decode planning: unpack split metadata into per-unit records, build the
// slot -> (symbol, f, slot - F) decode table, lay out the device workspace and
// launch the decode kernels.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "plan.hpp"
#include "../device/unpack.hpp"

namespace recoil {

namespace {
constexpr size_t kAlign = kWsAlign;
inline size_t align_up(size_t v) { return ws_align(v); }
}  // namespace

// Build the per-unit records of Sec. 4.1: unit u (0-based) starts at split
// point u+1 or, for the last unit, at the final states; it decodes groups
// top .. glo and stores ghi .. glo, where ghi is the group of its own
// synchronisation completion point (all lanes switched on) and glo is one
// above the previous unit's.
recoil_status check_gpu_limits(const BlobData &b) {
    const uint32_t W = b.lanes, n = b.quant_bits;
    if (W != 32 && W != 64) return fail(RECOIL_ERR_UNSUPPORTED, "plan: GPU decoding needs W = 32 or 64");
    // Eq. 2 is evaluated with a 24-bit multiply, f (x >> n): x >> n fits 24 bits only for n >= 8.
    if (n < 8 || n > 16) return fail(RECOIL_ERR_UNSUPPORTED, "plan: GPU decoding needs 8 <= n <= 16");
    if (b.n_symbols >= (1ull << 32) || b.n_words() + kChunkPadWords >= (1ull << 31))
        return fail(RECOIL_ERR_UNSUPPORTED, "plan: N must be below 2^32 and B below 2^31 - 1024 words");
    if (b.symbol_bytes == 2 && b.alphabet > 65536) return fail(RECOIL_ERR_UNSUPPORTED, "plan: alphabet too large");
    if (b.adaptive && (n > 12 || b.symbol_bytes != 1 || ((uint64_t)b.tables << (n + 2)) > kMaxAdaptiveTableBytes))
        return fail(RECOIL_ERR_UNSUPPORTED,
                    "plan: adaptive decoding needs uint8 symbols, n <= 12 and tables x 2^n x 4 <= 64 KiB");
    if (n > 12 && wide_ranks(b) > kMaxWideRanks)
        return fail(RECOIL_ERR_UNSUPPORTED, "plan: n > 12 decoding needs at most 4096 symbols with f > 0");
    return RECOIL_OK;
}

uint32_t wide_ranks(const BlobData &b) {
    uint32_t r = 0;
    for (uint32_t s = 0; s < b.alphabet; ++s) r += b.freq[s] != 0;
    return r;
}

recoil_status build_units(const std::shared_ptr<const BlobData> &bp, PlanData &pl) {
    const BlobData &b = *bp;
    const uint32_t W = b.lanes, M = b.splits();
    if (recoil_status st = check_gpu_limits(b)) return st;
    pl.blob = bp;
    pl.units = M;
    // Default launch shape: waves per workgroup chosen at launch (16, or 1 for
    // launches with few runs), 8-group super-steps when the table is small enough
    // for two 16-wave workgroups per CU (uint8 symbols), 4-group otherwise.
    pl.tuning.waves = 0;
    pl.tuning.chunk_groups = default_chunk_groups(b);
    pl.tuning.blocks_per_cu = 0;
    const uint64_t G = b.groups();
    pl.meta.resize(M);
    pl.lanes.resize((size_t)M * W);
    if (b.partitioned()) {
        // Conventional sub-sequences (Sec. 2.3): unit u decodes sub-sequence u alone,
        // from its final states over its own words, groups glo .. top.
        for (uint32_t u = 0; u < M; ++u) {
            UnitMeta &m = pl.meta[u];
            const uint64_t lo = (uint64_t)u * b.part_size, hi = std::min<uint64_t>(b.n_symbols, lo + b.part_size);
            m.glo = (uint32_t)(lo / W);
            m.top = hi > lo ? (uint32_t)((hi - 1) / W) : m.glo;
            m.ghi = m.top;
            m.next = (uint32_t)(u + 1 < M ? b.part_start[u + 1] : b.n_words());
            for (uint32_t j = 0; j < W; ++j) pl.lanes[(size_t)u * W + j] = b.part_final[(size_t)u * W + j];
        }
        return RECOIL_OK;
    }
    uint32_t prev_sync = 0;
    for (uint32_t u = 0; u < M; ++u) {
        UnitMeta &m = pl.meta[u];
        m.glo = (u == 0) ? 0u : prev_sync + 1;
        if (u + 1 == M) {
            m.next = (uint32_t)b.n_words();
            m.top = G ? (uint32_t)(G - 1) : 0u;
            m.ghi = m.top;
            for (uint32_t j = 0; j < W; ++j) pl.lanes[(size_t)u * W + j] = b.final_states[j];
        } else {
            const uint64_t k = u;   // split point u+1 is stored at index u
            m.next = (uint32_t)b.sp_next[k];
            m.top = (uint32_t)b.sp_anchor[k];
            uint32_t maxdiff = 0;
            for (uint32_t j = 0; j < W; ++j) {
                const uint32_t d = b.sp_gdiff[k * W + j];
                maxdiff = std::max(maxdiff, d);
                pl.lanes[(size_t)u * W + j] = (uint32_t)b.sp_state[k * W + j] | (d << 16);
            }
            m.ghi = m.top - maxdiff;     // group where every lane has been switched on
            prev_sync = m.ghi;
        }
    }
    return RECOIL_OK;
}

namespace {
inline uint32_t bit_length(uint64_t v) { return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u; }
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return b ? (a + b - 1) / b : 0; }
}  // namespace

// The per-unit records of the blob obtained by combining `full` to `target`
// units (every ceil(M/target)-th split point kept, Sec. 3.3), built in one pass
// over the kept split points without materialising the combined blob.
// *packed_bytes receives the size of that blob's packed metadata section (the
// series of Sec. 4.3: signed offset and group series, then per split point W
// 16-bit states and an unsigned group-difference series).
recoil_status build_units_combined(const std::shared_ptr<const BlobData> &bp, uint32_t target, PlanData &pl,
                                   uint64_t *packed_bytes) {
    const BlobData &b = *bp;
    const uint32_t W = b.lanes, M = b.splits();
    if (b.partitioned()) return fail(RECOIL_ERR_UNSUPPORTED, "combine: sub-sequences cannot be merged");
    if (recoil_status st = check_gpu_limits(b)) return st;
    const uint32_t step = (uint32_t)ceil_div(M, std::min(std::max(target, 1u), M));
    const uint32_t Mc = (M - 1) / step + 1;
    pl.blob = bp;
    pl.units = Mc;
    pl.tuning.waves = 0;
    pl.tuning.chunk_groups = default_chunk_groups(b);
    pl.tuning.blocks_per_cu = 0;
    const uint64_t G = b.groups();
    pl.meta.resize(Mc);
    pl.lanes.resize((size_t)Mc * W);
    const uint64_t Eb = ceil_div(b.n_words(), Mc), Eg = ceil_div(G, Mc);
    uint64_t max_o = 0, max_x = 0, bits = 0;
    uint32_t prev_sync = 0;
    for (uint32_t u = 0; u < Mc; ++u) {
        UnitMeta &m = pl.meta[u];
        m.glo = (u == 0) ? 0u : prev_sync + 1;
        uint32_t *lanes = &pl.lanes[(size_t)u * W];
        if (u + 1 == Mc) {
            m.next = (uint32_t)b.n_words();
            m.top = G ? (uint32_t)(G - 1) : 0u;
            m.ghi = m.top;
            for (uint32_t j = 0; j < W; ++j) lanes[j] = b.final_states[j];
            continue;
        }
        const uint64_t k = (uint64_t)(u + 1) * step - 1;   // split point (u+1)*step, stored at index - 1
        m.next = (uint32_t)b.sp_next[k];
        m.top = (uint32_t)b.sp_anchor[k];
        const uint16_t *st = &b.sp_state[k * W];
        const uint16_t *gd = &b.sp_gdiff[k * W];
        uint32_t maxdiff = 0;
        for (uint32_t j = 0; j < W; ++j) {
            maxdiff = std::max<uint32_t>(maxdiff, gd[j]);
            lanes[j] = (uint32_t)st[j] | ((uint32_t)gd[j] << 16);
        }
        m.ghi = m.top - maxdiff;
        prev_sync = m.ghi;
        const int64_t o = (int64_t)b.sp_next[k] - (int64_t)((u + 1) * Eb);
        const int64_t x = (int64_t)(b.sp_anchor[k] + 1) - (int64_t)((u + 1) * Eg);
        max_o = std::max<uint64_t>(max_o, o < 0 ? (uint64_t)-o : (uint64_t)o);
        max_x = std::max<uint64_t>(max_x, x < 0 ? (uint64_t)-x : (uint64_t)x);
        bits += 16ull * W + 4 + (uint64_t)W * std::max<uint32_t>(1, bit_length(maxdiff));
    }
    if (Mc > 1) {
        const uint32_t wo = std::max<uint32_t>(1, bit_length(max_o)), wx = std::max<uint32_t>(1, bit_length(max_x));
        if (wo > 32 || wx > 32) return fail(RECOIL_ERR_INFEASIBLE, "combine: metadata does not fit its series");
        bits += 2ull * 5 + (uint64_t)(Mc - 1) * (2 + wo + wx);
    }
    if (packed_bytes) *packed_bytes = (bits + 7) / 8;
    return RECOIL_OK;
}

// Wide decode table (13 <= n <= 16): 16-slot buckets, then one entry per symbol
// with f > 0 (layout in decode.hpp).
void build_wide_table(const BlobData &b, PlanData &pl) {
    const uint32_t n = b.quant_bits, buckets = 1u << (n - 4);
    std::vector<uint32_t> bucket(buckets, 0);
    std::vector<uint32_t> ranks;
    uint32_t F = 0, r = 0;
    for (uint32_t s = 0; s < b.alphabet; ++s) {
        const uint32_t f = b.freq[s];
        if (!f) continue;
        // Symbol s holds slots F .. F+f-1: it is the first of every bucket it covers
        // from the start, and marks its start inside the bucket holding slot F.
        if (F % 16) bucket[F / 16] |= 1u << (F % 16 - 1);
        for (uint32_t q = (F + 15) / 16; q * 16 < F + f; ++q) bucket[q] |= r << 16;
        ranks.push_back(f);
        ranks.push_back(s | (F << 16));
        F += f;
        ++r;
    }
    const size_t bytes = 4 * (size_t)buckets + 4 * ranks.size();
    pl.lut.assign((bytes + 15) / 16 * 16, 0);
    std::memcpy(pl.lut.data(), bucket.data(), 4 * (size_t)buckets);
    std::memcpy(pl.lut.data() + 4 * (size_t)buckets, ranks.data(), 4 * ranks.size());
}

// Decode table: slot -> (symbol, f, slot - F) for the 2^n slots (Eq. 2).
void build_table(const BlobData &b, PlanData &pl) {
    const uint32_t slots = 1u << b.quant_bits;
    uint32_t present = 0, only = 0;
    for (uint32_t s = 0; s < b.alphabet; ++s)
        if (b.freq[s]) { ++present; only = s; }
    pl.single_symbol = present == 1 && !b.adaptive;
    pl.fill_symbol = only;
    if (b.quant_bits > 12) {
        build_wide_table(b, pl);
        return;
    }
    const size_t esz = b.symbol_bytes == 1 ? 4 : 8;
    // Adaptive coding: the tables' decode tables end to end, table t at slot t 2^n.
    pl.lut.assign((size_t)slots * esz * b.tables, 0);
    for (uint32_t t = 0; t < b.tables; ++t) {
    uint32_t F = 0;
    for (uint32_t s = 0; s < b.alphabet; ++s) {
        const uint32_t f = b.freq[(size_t)t * b.alphabet + s];
        for (uint32_t r = 0; r < f; ++r) {
            const uint32_t slot = t * slots + F + r;
            if (b.symbol_bytes == 1) {
                const uint32_t e = s | ((f & 0xFFFu) << 8) | (r << 20);
                std::memcpy(&pl.lut[(size_t)slot * 4], &e, 4);
            } else {
                const uint32_t e0 = f | (r << 16), e1 = s;
                std::memcpy(&pl.lut[(size_t)slot * 8], &e0, 4);
                std::memcpy(&pl.lut[(size_t)slot * 8 + 4], &e1, 4);
            }
        }
        F += f;
    }
    }
}

recoil_status build_plan(const std::shared_ptr<const BlobData> &bp, PlanData &pl) {
    recoil_status st = build_units(bp, pl);
    if (st) return st;
    build_table(*bp, pl);
    size_t off = 0;
    pl.off_words = off; off += words_section_bytes(bp->n_words());
    pl.off_lut = off;   off = align_up(off + pl.lut.size());
    pl.off_meta = off;  off = align_up(off + pl.meta.size() * sizeof(UnitMeta));
    pl.off_lanes = off; off = align_up(off + pl.lanes.size() * 4);
    pl.total = off;
    return RECOIL_OK;
}

recoil_status build_plan_packed(const std::shared_ptr<const BlobData> &bp, uint32_t target, PlanData &pl) {
    const BlobData &b = *bp;
    if (b.partitioned()) return fail(RECOIL_ERR_UNSUPPORTED, "plan_create_packed: sub-sequence records are not packed");
    if (recoil_status st = check_gpu_limits(b)) return st;
    const uint32_t M = b.splits(), W = b.lanes;
    if (b.block_bit.size() + 1 != M || 8ull * b.meta_bits.size() >= (1ull << 32))
        return fail(RECOIL_ERR_UNSUPPORTED, "plan_create_packed: metadata section above 2^32 bits");
    pl.blob = bp;
    pl.packed = true;
    pl.step = (uint32_t)ceil_div(M, target == 0 ? M : std::min(target, M));
    pl.units = (M - 1) / pl.step + 1;
    pl.tuning.waves = 0;
    pl.tuning.chunk_groups = default_chunk_groups(b);
    pl.tuning.blocks_per_cu = 0;
    pl.packed_bits.assign(b.meta_bits.size() + 8, 0);
    std::copy(b.meta_bits.begin(), b.meta_bits.end(), pl.packed_bits.begin());
    pl.block_bit.assign(b.block_bit.begin(), b.block_bit.end());
    build_table(b, pl);
    size_t off = 0;
    pl.off_words = off;  off += words_section_bytes(b.n_words());
    pl.off_lut = off;    off = align_up(off + pl.lut.size());
    pl.off_meta = off;   off = align_up(off + (size_t)pl.units * sizeof(UnitMeta));
    pl.off_lanes = off;  off = align_up(off + (size_t)pl.units * W * 4);
    pl.off_bits = off;   off = align_up(off + pl.packed_bits.size());
    pl.off_blocks = off; off = align_up(off + pl.block_bit.size() * 4);
    pl.off_final = off;  off = align_up(off + (size_t)W * 4);
    pl.total = off;
    return RECOIL_OK;
}

}  // namespace recoil

struct recoil_plan {
    recoil::PlanData d;
};

namespace {

// The unpack kernel of a packed plan, reading the sections already in the workspace.
hipError_t enqueue_unpack(const recoil::PlanData &pl, char *base, hipStream_t stream) {
    using namespace recoil;
    const BlobData &b = *pl.blob;
    UnpackParams u{};
    u.bits = reinterpret_cast<const uint8_t *>(base + pl.off_bits);
    u.block_bit = reinterpret_cast<const uint32_t *>(base + pl.off_blocks);
    u.final_states = reinterpret_cast<const uint32_t *>(base + pl.off_final);
    u.meta = reinterpret_cast<UnitMeta *>(base + pl.off_meta);
    u.lanes = reinterpret_cast<uint32_t *>(base + pl.off_lanes);
    u.words = b.n_words();
    u.groups = b.groups();
    u.splits = b.splits();
    u.eb = (u.words + u.splits - 1) / u.splits;
    u.eg = (u.groups + u.splits - 1) / u.splits;
    u.step = pl.step;
    u.units = pl.units;
    u.lanes_per_unit = b.lanes;
    return launch_unpack(u, stream);
}

}  // namespace

extern "C" {

recoil_status recoil_plan_create(const recoil_blob *blob, recoil_plan **out, size_t *device_bytes) {
    return recoil::guarded("plan_create", [&]() -> recoil_status {
    using namespace recoil;
    if (!blob || !out) return fail(RECOIL_ERR_INVALID_ARG, "plan_create: bad arguments");
    *out = nullptr;
    std::unique_ptr<recoil_plan> p(new recoil_plan());
    recoil_status st = build_plan(blob->data, p->d);
    if (st) return st;
    if (device_bytes) *device_bytes = p->d.total;
    *out = p.release();
    return RECOIL_OK;
    });
}

recoil_status recoil_plan_create_packed(const recoil_blob *blob, uint32_t target_units, recoil_plan **out,
                                        size_t *device_bytes) {
    return recoil::guarded("plan_create_packed", [&]() -> recoil_status {
    using namespace recoil;
    if (!blob || !out) return fail(RECOIL_ERR_INVALID_ARG, "plan_create_packed: bad arguments");
    *out = nullptr;
    std::unique_ptr<recoil_plan> p(new recoil_plan());
    recoil_status st = build_plan_packed(blob->data, target_units, p->d);
    if (st) return st;
    if (device_bytes) *device_bytes = p->d.total;
    *out = p.release();
    return RECOIL_OK;
    });
}

size_t recoil_plan_metadata_device_bytes(const recoil_plan *plan) {
    if (!plan) return 0;
    const recoil::PlanData &pl = plan->d;
    if (pl.packed) return pl.blob->meta_bits.size() + pl.block_bit.size() * 4 + (size_t)pl.blob->lanes * 4;
    return pl.meta.size() * sizeof(recoil::UnitMeta) + pl.lanes.size() * 4;
}

recoil_status recoil_plan_decode_table(const recoil_plan *plan, void *dst, size_t cap, size_t *bytes) {
    using namespace recoil;
    if (!plan) return fail(RECOIL_ERR_INVALID_ARG, "plan_decode_table: NULL plan");
    const std::vector<uint8_t> &t = plan->d.lut;
    if (bytes) *bytes = t.size();
    if (!dst) return RECOIL_OK;
    if (cap < t.size()) return fail(RECOIL_ERR_BUFFER_TOO_SMALL, "plan_decode_table: buffer too small");
    std::memcpy(dst, t.data(), t.size());
    return RECOIL_OK;
}

recoil_status recoil_plan_get_layout(const recoil_plan *plan, recoil_plan_layout *out) {
    using namespace recoil;
    if (!plan || !out) return fail(RECOIL_ERR_INVALID_ARG, "plan_get_layout: bad arguments");
    const PlanData &pl = plan->d;
    *out = recoil_plan_layout{pl.off_words, pl.off_lut, pl.off_meta, pl.off_lanes, pl.total, pl.units,
                              pl.blob->lanes, pl.packed ? 1u : 0u};
    return RECOIL_OK;
}

recoil_status recoil_plan_upload(const recoil_plan *plan, void *d_ws, size_t bytes, hipStream_t stream) {
    return recoil::guarded("plan_upload", [&]() -> recoil_status {
    using namespace recoil;
    if (!plan || !d_ws) return fail(RECOIL_ERR_INVALID_ARG, "plan_upload: bad arguments");
    const PlanData &pl = plan->d;
    if (bytes < pl.total) return fail(RECOIL_ERR_BUFFER_TOO_SMALL, "plan_upload: workspace too small");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(RECOIL_ERR_ALIGNMENT, "plan_upload: workspace not 256-byte aligned");
    char *base = static_cast<char *>(d_ws);
    const BlobData &b = *pl.blob;
    hipError_t e = hipSuccess;
    if (b.n_words()) e = stage_h2d(base + pl.off_words, b.words(), 2 * b.n_words(), stream);
    if (e == hipSuccess) e = stage_h2d(base + pl.off_lut, pl.lut.data(), pl.lut.size(), stream);
    if (pl.packed) {
        // The packed section, block offsets and final states, then the unpacker
        // writes the unit and lane records on the same stream.
        if (e == hipSuccess) e = stage_h2d(base + pl.off_bits, pl.packed_bits.data(), pl.packed_bits.size(), stream);
        if (e == hipSuccess && !pl.block_bit.empty())
            e = stage_h2d(base + pl.off_blocks, pl.block_bit.data(), pl.block_bit.size() * 4, stream);
        if (e == hipSuccess) e = stage_h2d(base + pl.off_final, b.final_states.data(), (size_t)b.lanes * 4, stream);
        if (e == hipSuccess) e = enqueue_unpack(pl, base, stream);
    } else {
        if (e == hipSuccess) e = stage_h2d(base + pl.off_meta, pl.meta.data(), pl.meta.size() * sizeof(UnitMeta), stream);
        if (e == hipSuccess) e = stage_h2d(base + pl.off_lanes, pl.lanes.data(), pl.lanes.size() * 4, stream);
    }
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("plan_upload: ") + hipGetErrorString(e));
    return RECOIL_OK;
    });
}

recoil_status recoil_plan_unpack(const recoil_plan *plan, void *d_ws, hipStream_t stream) {
    using namespace recoil;
    if (!plan || !d_ws) return fail(RECOIL_ERR_INVALID_ARG, "plan_unpack: bad arguments");
    if (!plan->d.packed) return fail(RECOIL_ERR_INVALID_ARG, "plan_unpack: not a packed plan");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(RECOIL_ERR_ALIGNMENT, "plan_unpack: workspace not 256-byte aligned");
    hipError_t e = enqueue_unpack(plan->d, static_cast<char *>(d_ws), stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("plan_unpack: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

void recoil_plan_free(recoil_plan *plan) { delete plan; }

recoil_status recoil_plan_set_tuning(recoil_plan *plan, const recoil_tuning *t) {
    using namespace recoil;
    if (!plan || !t) return fail(RECOIL_ERR_INVALID_ARG, "plan_set_tuning: bad arguments");
    const bool ok = (t->waves == 0 || t->waves == 1 || t->waves == 8 || t->waves == 16) &&
                    (t->chunk_groups == 4 || t->chunk_groups == 8);
    if (!ok) return fail(RECOIL_ERR_INVALID_ARG, "plan_set_tuning: unsupported shape");
    plan->d.tuning.waves = t->waves;
    plan->d.tuning.chunk_groups = t->chunk_groups;
    plan->d.tuning.blocks_per_cu = t->blocks_per_cu;
    plan->d.tuning.units_per_run = t->units_per_run;
    return RECOIL_OK;
}

namespace {

recoil::DecodeParams decode_params(const recoil::PlanData &pl, const void *d_ws, void *d_out, uint32_t *d_error) {
    using namespace recoil;
    const BlobData &b = *pl.blob;
    const char *base = static_cast<const char *>(d_ws);
    DecodeParams p{};
    p.words = reinterpret_cast<const uint16_t *>(base + pl.off_words);
    p.lut = base + pl.off_lut;
    p.meta = reinterpret_cast<const UnitMeta *>(base + pl.off_meta);
    p.lanes = reinterpret_cast<const uint32_t *>(base + pl.off_lanes);
    p.out = d_out;
    p.err = d_error;
    p.n_symbols = b.n_symbols;
    p.units = pl.units;
    p.run = 1;
    p.runs = p.units;
    p.quant_bits = b.quant_bits;
    p.fill_symbol = pl.fill_symbol;
    p.single_symbol = pl.single_symbol ? 1u : 0u;
    p.partitioned = b.partitioned() ? 1u : 0u;
    p.tables = b.tables;
    p.lut_bytes = (uint32_t)pl.lut.size();
    p.tidx = nullptr;
    return p;
}

}  // namespace

recoil_status recoil_decode(const recoil_plan *plan, const void *d_ws, void *d_out, uint32_t *d_error,
                            hipStream_t stream) {
    using namespace recoil;
    if (!plan || !d_ws || !d_error || (!d_out && plan->d.blob->n_symbols))
        return fail(RECOIL_ERR_INVALID_ARG, "decode: bad arguments");
    if (reinterpret_cast<uintptr_t>(d_out) % 16 || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(RECOIL_ERR_ALIGNMENT, "decode: output must be 16-byte and workspace 256-byte aligned");
    const PlanData &pl = plan->d;
    if (pl.blob->adaptive && pl.blob->n_symbols)
        return fail(RECOIL_ERR_INVALID_ARG, "decode: an adaptive stream needs its table index (recoil_decode_adaptive)");
    const DecodeParams p = decode_params(pl, d_ws, d_out, d_error);
    hipError_t e = launch_decode(p, pl.blob->lanes, pl.blob->symbol_bytes, pl.tuning, stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

recoil_status recoil_decode_adaptive(const recoil_plan *plan, const void *d_ws, const uint8_t *d_table_index,
                                     void *d_out, uint32_t *d_error, hipStream_t stream) {
    using namespace recoil;
    if (!plan || !d_ws || !d_error || ((!d_out || !d_table_index) && plan->d.blob->n_symbols))
        return fail(RECOIL_ERR_INVALID_ARG, "decode_adaptive: bad arguments");
    if (!plan->d.blob->adaptive) return fail(RECOIL_ERR_INVALID_ARG, "decode_adaptive: not an adaptive stream");
    if (reinterpret_cast<uintptr_t>(d_out) % 16 || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(RECOIL_ERR_ALIGNMENT, "decode_adaptive: output must be 16-byte and workspace 256-byte aligned");
    const PlanData &pl = plan->d;
    DecodeParams p = decode_params(pl, d_ws, d_out, d_error);
    p.tidx = d_table_index;
    hipError_t e = launch_decode(p, pl.blob->lanes, pl.blob->symbol_bytes, pl.tuning, stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode_adaptive: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

recoil_status recoil_decode_count_writes(const recoil_plan *plan, const void *d_ws, void *d_out, uint32_t *d_counts,
                                        uint32_t *d_error, hipStream_t stream) {
    using namespace recoil;
    if (!plan || !d_ws || !d_error || ((!d_out || !d_counts) && plan->d.blob->n_symbols))
        return fail(RECOIL_ERR_INVALID_ARG, "decode_count_writes: bad arguments");
    if (reinterpret_cast<uintptr_t>(d_out) % 16 || reinterpret_cast<uintptr_t>(d_ws) % kAlign ||
        reinterpret_cast<uintptr_t>(d_counts) % 4)
        return fail(RECOIL_ERR_ALIGNMENT, "decode_count_writes: misaligned buffer");
    const PlanData &pl = plan->d;
    if (pl.single_symbol) return fail(RECOIL_ERR_UNSUPPORTED, "decode_count_writes: single-symbol stream (no decode kernel)");
    if (pl.blob->adaptive) return fail(RECOIL_ERR_UNSUPPORTED, "decode_count_writes: adaptive stream");
    DecodeParams p = decode_params(pl, d_ws, d_out, d_error);
    p.counts = d_counts;
    hipError_t e = launch_decode(p, pl.blob->lanes, pl.blob->symbol_bytes, pl.tuning, stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode_count_writes: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

recoil_status recoil_plan_units(const recoil_plan *plan, uint32_t *records, uint32_t cap, uint32_t *count) {
    using namespace recoil;
    if (!plan) return fail(RECOIL_ERR_INVALID_ARG, "plan_units: NULL plan");
    const std::vector<UnitMeta> &m = plan->d.meta;
    if (count) *count = plan->d.units;
    if (!records) return RECOIL_OK;
    if (plan->d.packed) return fail(RECOIL_ERR_UNSUPPORTED, "plan_units: a packed plan's records exist on the device only");
    if (cap < m.size()) return fail(RECOIL_ERR_BUFFER_TOO_SMALL, "plan_units: records too small");
    for (size_t u = 0; u < m.size(); ++u) {
        records[4 * u + 0] = m[u].next;
        records[4 * u + 1] = m[u].top;
        records[4 * u + 2] = m[u].ghi;
        records[4 * u + 3] = m[u].glo;
    }
    return RECOIL_OK;
}

recoil_status recoil_plan_shape(const recoil_plan *plan, recoil_decode_shape *out) {
    using namespace recoil;
    if (!plan || !out) return fail(RECOIL_ERR_INVALID_ARG, "plan_shape: bad arguments");
    const PlanData &pl = plan->d;
    DecodeShape sh{};
    hipError_t e = launch_decode(decode_params(pl, nullptr, nullptr, nullptr), pl.blob->lanes, pl.blob->symbol_bytes,
                                 pl.tuning, nullptr, &sh);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("plan_shape: ") + hipGetErrorString(e));
    *out = recoil_decode_shape{sh.blocks, sh.waves, sh.units_per_run, sh.runs, sh.units_per_wave};
    return RECOIL_OK;
}

namespace {
std::mutex g_plan_tune_mu;
std::map<std::string, recoil::DecodeTuning> g_plan_tune_cache;
}  // namespace

recoil_status recoil_plan_autotune(recoil_plan *plan, void *d_ws, void *d_out, uint32_t *d_error, hipStream_t stream,
                                   uint32_t reps, recoil_tuning *best_out, float *best_ms) {
    using namespace recoil;
    if (!plan || !d_ws || !d_error || reps == 0 || (!d_out && plan->d.blob->n_symbols))
        return fail(RECOIL_ERR_INVALID_ARG, "plan_autotune: bad arguments");
    PlanData &pl = plan->d;
    const BlobData &b = *pl.blob;
    if (b.adaptive) return fail(RECOIL_ERR_UNSUPPORTED, "plan_autotune: adaptive streams keep the default shape");
    auto report = [&](const DecodeTuning &t, float ms) {
        if (best_out) *best_out = recoil_tuning{t.waves, t.chunk_groups, 1, t.blocks_per_cu, t.units_per_run};
        if (best_ms) *best_ms = ms;
    };
    hipDeviceProp_t prop{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    const std::string key = std::string(prop.gcnArchName) + "/" + std::to_string(b.n_symbols) + "/" +
                            std::to_string(pl.units) + "/" + std::to_string(b.lanes) + "/" +
                            std::to_string(b.symbol_bytes) + "/" + std::to_string(b.quant_bits);
    {
        std::lock_guard<std::mutex> lk(g_plan_tune_mu);
        auto it = g_plan_tune_cache.find(key);
        if (it != g_plan_tune_cache.end()) {
            pl.tuning = it->second;
            report(it->second, -1.0f);
            return RECOIL_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RECOIL_ERR_HIP, "plan_autotune: event creation failed");
    const DecodeTuning saved = pl.tuning;
    DecodeTuning best = saved;
    float best_t = 1e30f;
    const uint32_t waves_opts[] = {1, 8, 16}, k_opts[] = {4, 8}, run_opts[] = {0, 1, 2, 4};
    for (uint32_t w : waves_opts)
        for (uint32_t k : k_opts)
            for (uint32_t r : run_opts) {
                pl.tuning = DecodeTuning{w, k, 0, r};
                // One warm-up launch, then the median of `reps` timed launches.
                if (recoil_decode(plan, d_ws, d_out, d_error, stream)) continue;
                std::vector<float> ts;
                for (uint32_t i = 0; i < reps; ++i) {
                    (void)hipEventRecord(e0, stream);
                    (void)recoil_decode(plan, d_ws, d_out, d_error, stream);
                    (void)hipEventRecord(e1, stream);
                    (void)hipEventSynchronize(e1);
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ts.push_back(ms);
                }
                std::sort(ts.begin(), ts.end());
                const float med = ts[ts.size() / 2];
                if (med < best_t) { best_t = med; best = pl.tuning; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_t >= 1e30f) {
        pl.tuning = saved;
        return fail(RECOIL_ERR_HIP, "plan_autotune: no configuration ran");
    }
    pl.tuning = best;
    {
        std::lock_guard<std::mutex> lk(g_plan_tune_mu);
        g_plan_tune_cache[key] = best;
    }
    report(best, best_t);
    return RECOIL_OK;
}

}  // extern "C"
