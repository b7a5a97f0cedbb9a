// Batched decoding of many independent Recoil streams: host planning, device
// layout, the persistent launch, the one-launch-per-stream baseline, HIP graph
// capture and the autotuner.
#include <algorithm>
#include <memory>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../device/batch.hpp"
#include "plan.hpp"
#include "recoil_batch.h"

namespace recoil {

// Streams are split into classes by decode table, each decoded by a launch of its
// own whose LDS holds only its class's largest table: a 32 KiB uint16 table would
// otherwise halve the resident waves of every uint8 stream's launch. Class 2 holds
// the two-level tables of 13 <= n <= 16, decoded by a kernel of their own.
constexpr uint32_t kBatchClasses = 3, kWideClass = 2;
constexpr uint32_t kSmallTableBytes = 16384;   // class 0: tables up to 16 KiB (uint8, n <= 12)
inline uint32_t table_class(const PlanData &pl) {
    if (pl.blob->quant_bits > 12) return kWideClass;
    return pl.lut.size() <= kSmallTableBytes ? 0u : 1u;
}

struct BatchData {
    std::vector<PlanData> plans;
    std::vector<StreamDesc> descs;
    std::vector<WorkItem> items;               // class 0's items, then class 1's, then class 2's
    std::vector<uint64_t> out_off, out_bytes;
    size_t off_head = 0, off_descs = 0, off_items = 0, items_cap = 0, total_ws = 0, total_out = 0;
    uint32_t lut_bytes = 0;                    // largest table of the batch
    uint32_t cls_lut[kBatchClasses] = {};      // largest table of each class
    uint32_t cls_begin[kBatchClasses] = {}, cls_count[kBatchClasses] = {};
    recoil_tuning tuning{};
};

namespace {

// Head section of the batch workspace: one work-queue head per class (128 bytes
// apart), each reset by a kernel before its class's persistent launch.
constexpr size_t kHeadStride = 128, kBatchHeadBytes = kBatchClasses * kHeadStride;

// Units per run for a stream of M units under tuning value k (0 or 1: one).
uint32_t run_of(uint32_t M, uint32_t k) { return std::max(1u, std::min(k, std::max(M, 1u))); }

uint32_t pairs_of(const PlanData &pl, uint32_t k) {
    const uint32_t W = pl.blob->lanes, M = pl.blob->splits(), run = run_of(M, k);
    const uint32_t runs = (M + run - 1) / run;
    return W == 32 ? (runs + 1) / 2 : runs;
}

// Units per run of one stream: the tuned length, shortened for a stream with too
// few units to give each unit slot of a workgroup (waves x units per wave) a run
// of that length, so that its units spread over the waves instead of leaving
// some idle while others decode long runs.
uint32_t stream_run(const PlanData &pl, const recoil_tuning &t) {
    const uint32_t M = pl.blob->splits();
    if (pl.blob->partitioned()) return 1;   // independent sub-sequences: one unit per run
    const uint32_t slots = std::max(1u, t.waves * (pl.blob->lanes == 32 ? 2u : 1u));
    const uint32_t spread = std::max(1u, (M + slots - 1) / slots);
    return run_of(M, std::min(std::max(t.units_per_run, 1u), spread));
}

// Work items: per stream, waves * pairs_per_wave consecutive pairs each; streams
// in decreasing size so the longest work starts first.
void build_items(BatchData &b) {
    b.items.clear();
    std::vector<uint32_t> order(b.plans.size());
    for (uint32_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) {
        const uint32_t ca = table_class(b.plans[a]), cc = table_class(b.plans[c]);
        if (ca != cc) return ca < cc;
        return b.plans[a].blob->n_symbols * b.plans[a].blob->symbol_bytes >
               b.plans[c].blob->n_symbols * b.plans[c].blob->symbol_bytes;
    });
    const uint32_t per_item = std::max(1u, b.tuning.waves * b.tuning.pairs_per_wave);
    for (uint32_t c = 0; c < kBatchClasses; ++c) { b.cls_begin[c] = 0; b.cls_count[c] = 0; b.cls_lut[c] = 0; }
    for (uint32_t s : order) {
        const PlanData &pl = b.plans[s];
        if (pl.blob->n_symbols == 0) continue;
        const uint32_t c = table_class(pl);
        if (b.cls_count[c] == 0) b.cls_begin[c] = (uint32_t)b.items.size();
        b.cls_lut[c] = std::max<uint32_t>(b.cls_lut[c], (uint32_t)pl.lut.size());
        const size_t before = b.items.size();
        if (pl.single_symbol) {
            b.items.push_back({s, 0, 1, 1});
        } else {
            const uint32_t run = stream_run(pl, b.tuning);
            // A W = 32 stream with no more runs than a workgroup has waves decodes one
            // unit per wave (each run a wave of its own, not half of one).
            const uint32_t M = pl.blob->splits(), runs = (M + run - 1) / run;
            const bool single = pl.blob->lanes == 32 && runs <= b.tuning.waves;
            const uint32_t pairs = single ? runs : pairs_of(pl, run);
            const uint32_t tag = run | (single ? kItemSingle : 0u);
            for (uint32_t f = 0; f < pairs; f += per_item) b.items.push_back({s, f, std::min(per_item, pairs - f), tag});
        }
        b.cls_count[c] += (uint32_t)(b.items.size() - before);
    }
}

bool tuning_ok(const recoil_tuning &t) {
    return (t.waves == 8 || t.waves == 16) && (t.chunk_groups == 4 || t.chunk_groups == 8) && t.pairs_per_wave >= 1 &&
           t.pairs_per_wave <= 64 && t.units_per_run <= 64;
}

BatchTuning device_tuning(const recoil_tuning &t) { return BatchTuning{t.waves, t.chunk_groups, t.blocks_per_cu}; }

BatchParams params_of(const BatchData &b, uint32_t cls, void *d_ws, void *d_out, uint32_t *d_err) {
    BatchParams bp{};
    unsigned char *ws = static_cast<unsigned char *>(d_ws);
    bp.ws = ws;
    bp.out = static_cast<unsigned char *>(d_out);
    bp.streams = reinterpret_cast<const StreamDesc *>(ws + b.off_descs);
    bp.items = reinterpret_cast<const WorkItem *>(ws + b.off_items) + b.cls_begin[cls];
    bp.head = reinterpret_cast<uint32_t *>(ws + b.off_head + cls * kHeadStride);
    bp.err = d_err;
    bp.n_items = b.cls_count[cls];
    bp.lut_bytes = b.cls_lut[cls];
    bp.wide = cls == kWideClass ? 1u : 0u;
    return bp;
}

// One persistent launch per table class that has work, in class order.
hipError_t launch_classes(const BatchData &b, void *d_ws, void *d_out, uint32_t *d_err, hipStream_t stream) {
    for (uint32_t c = 0; c < kBatchClasses; ++c) {
        if (b.cls_count[c] == 0) continue;
        hipError_t e = launch_batch(params_of(b, c, d_ws, d_out, d_err), device_tuning(b.tuning), stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Launch shape fits the CU for every class that has work.
bool shape_fits(const BatchData &b, const recoil_tuning &t) {
    for (uint32_t c = 0; c < kBatchClasses; ++c)
        if (b.cls_count[c] && batch_blocks_per_cu(device_tuning(t), b.cls_lut[c], c == kWideClass) < 1) return false;
    return true;
}


std::mutex g_tune_mu;
std::map<std::string, recoil_tuning> g_tune_cache;

}  // namespace
}  // namespace recoil

struct recoil_batch {
    recoil::BatchData d;
};

struct recoil_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

recoil_tuning recoil_default_tuning(void) { return recoil_tuning{16, 4, 2, 0, 0}; }

recoil_status recoil_batch_create(const recoil_blob *const *blobs, uint32_t count, const recoil_tuning *tuning,
                                  recoil_batch **out, size_t *workspace_bytes, size_t *output_bytes) {
    return recoil::guarded("batch_create", [&]() -> recoil_status {
    using namespace recoil;
    if (!blobs || !out || count == 0) return fail(RECOIL_ERR_INVALID_ARG, "batch_create: bad arguments");
    *out = nullptr;
    std::unique_ptr<recoil_batch> hp(new recoil_batch());
    recoil_batch *h = hp.get();
    BatchData &b = h->d;
    b.tuning = tuning ? *tuning : recoil_default_tuning();
    if (!tuning_ok(b.tuning)) { return fail(RECOIL_ERR_INVALID_ARG, "batch_create: unsupported tuning"); }
    b.plans.resize(count);
    for (uint32_t i = 0; i < count; ++i) {
        if (!blobs[i]) { return fail(RECOIL_ERR_INVALID_ARG, "batch_create: NULL blob"); }
        if (blobs[i]->data->adaptive) { return fail(RECOIL_ERR_UNSUPPORTED, "batch_create: adaptive streams are decoded alone"); }
        recoil_status st = build_plan(blobs[i]->data, b.plans[i]);
        if (st) { return st; }
        b.lut_bytes = std::max<uint32_t>(b.lut_bytes, (uint32_t)b.plans[i].lut.size());
    }
    // Item capacity: the finest tuning (8 waves, one pair per wave).
    size_t cap = 0;
    for (const PlanData &pl : b.plans) cap += pl.single_symbol ? 1 : (pairs_of(pl, 1) + 7) / 8;
    b.items_cap = std::max<size_t>(cap, 1);
    size_t off = 0;
    b.off_head = off;  off = ws_align(off + kBatchHeadBytes);
    b.off_descs = off; off = ws_align(off + count * sizeof(StreamDesc));
    b.off_items = off; off = ws_align(off + b.items_cap * sizeof(WorkItem));
    b.descs.resize(count);
    b.out_off.resize(count);
    b.out_bytes.resize(count);
    size_t out_off = 0;
    for (uint32_t i = 0; i < count; ++i) {
        PlanData &pl = b.plans[i];
        const BlobData &bd = *pl.blob;
        StreamDesc &d = b.descs[i];
        std::memset(&d, 0, sizeof(d));
        d.words_off = off; off += words_section_bytes(bd.n_words());
        d.lut_off = off;   off = ws_align(off + pl.lut.size());
        d.meta_off = off;  off = ws_align(off + pl.meta.size() * sizeof(UnitMeta));
        d.lanes_off = off; off = ws_align(off + pl.lanes.size() * 4);
        d.out_off = out_off;
        d.n_symbols = bd.n_symbols;
        d.units = bd.splits();
        d.quant_bits = (uint8_t)bd.quant_bits;
        d.symbol_bytes = (uint8_t)bd.symbol_bytes;
        d.lanes = (uint8_t)bd.lanes;
        d.single_symbol = pl.single_symbol ? 1 : 0;
        d.fill_symbol = pl.fill_symbol;
        d.partitioned = bd.partitioned() ? 1 : 0;
        d.lut_chunks = (uint16_t)(pl.lut.size() / 16);
        b.out_off[i] = out_off;
        b.out_bytes[i] = bd.n_symbols * bd.symbol_bytes;
        out_off = ws_align(out_off + b.out_bytes[i]);
    }
    b.total_ws = off;
    b.total_out = std::max<size_t>(out_off, 256);
    build_items(b);
    if (b.items.size() > b.items_cap) { return fail(RECOIL_ERR_INVALID_ARG, "batch_create: too many items"); }
    if (workspace_bytes) *workspace_bytes = b.total_ws;
    if (output_bytes) *output_bytes = b.total_out;
    *out = hp.release();
    return RECOIL_OK;
    });
}

void recoil_batch_free(recoil_batch *batch) { delete batch; }

recoil_status recoil_batch_output_offset(const recoil_batch *batch, uint32_t index, uint64_t *offset, uint64_t *bytes) {
    using namespace recoil;
    if (!batch || index >= batch->d.descs.size()) return fail(RECOIL_ERR_INVALID_ARG, "batch_output_offset: bad index");
    if (offset) *offset = batch->d.out_off[index];
    if (bytes) *bytes = batch->d.out_bytes[index];
    return RECOIL_OK;
}

uint32_t recoil_batch_items(const recoil_batch *batch) { return batch ? (uint32_t)batch->d.items.size() : 0; }

static recoil_status upload_items(const recoil::BatchData &b, void *d_ws, hipStream_t stream) {
    using namespace recoil;
    if (b.items.size() > b.items_cap) return fail(RECOIL_ERR_INVALID_ARG, "batch upload: too many items");
    char *base = static_cast<char *>(d_ws);
    hipError_t e = hipMemcpyAsync(base + b.off_items, b.items.data(), b.items.size() * sizeof(WorkItem),
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("batch upload: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

recoil_status recoil_batch_upload(const recoil_batch *batch, void *d_ws, size_t bytes, hipStream_t stream) {
    return recoil::guarded("batch_upload", [&]() -> recoil_status {
    using namespace recoil;
    if (!batch || !d_ws) return fail(RECOIL_ERR_INVALID_ARG, "batch_upload: bad arguments");
    const BatchData &b = batch->d;
    if (bytes < b.total_ws) return fail(RECOIL_ERR_BUFFER_TOO_SMALL, "batch_upload: workspace too small");
    if (reinterpret_cast<uintptr_t>(d_ws) % kWsAlign) return fail(RECOIL_ERR_ALIGNMENT, "batch_upload: workspace not 256-byte aligned");
    char *base = static_cast<char *>(d_ws);
    static const uint8_t zero_head[kBatchHeadBytes] = {};
    hipError_t e = hipMemcpyAsync(base + b.off_head, zero_head, kBatchHeadBytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + b.off_descs, b.descs.data(), b.descs.size() * sizeof(StreamDesc),
                           hipMemcpyHostToDevice, stream);
    for (size_t i = 0; e == hipSuccess && i < b.plans.size(); ++i) {
        const PlanData &pl = b.plans[i];
        const StreamDesc &d = b.descs[i];
        if (pl.blob->n_words())
            e = stage_h2d(base + d.words_off, pl.blob->words(), 2 * pl.blob->n_words(), stream);
        if (e == hipSuccess) e = stage_h2d(base + d.lut_off, pl.lut.data(), pl.lut.size(), stream);
        if (e == hipSuccess && !pl.meta.empty())
            e = stage_h2d(base + d.meta_off, pl.meta.data(), pl.meta.size() * sizeof(UnitMeta), stream);
        if (e == hipSuccess && !pl.lanes.empty())
            e = stage_h2d(base + d.lanes_off, pl.lanes.data(), pl.lanes.size() * 4, stream);
    }
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("batch_upload: ") + hipGetErrorString(e));
    return upload_items(b, d_ws, stream);
    });
}

recoil_status recoil_batch_set_tuning(recoil_batch *batch, const recoil_tuning *t, void *d_ws, hipStream_t stream) {
    using namespace recoil;
    if (!batch || !t || !tuning_ok(*t)) return fail(RECOIL_ERR_INVALID_ARG, "batch_set_tuning: unsupported tuning");
    const recoil_tuning old = batch->d.tuning;
    batch->d.tuning = *t;
    build_items(batch->d);
    if (batch->d.items.size() > batch->d.items_cap) {
        // Keep the batch as it was: its workspace holds items_cap items.
        batch->d.tuning = old;
        build_items(batch->d);
        return fail(RECOIL_ERR_INVALID_ARG, "batch_set_tuning: too many items");
    }
    if (d_ws) return upload_items(batch->d, d_ws, stream);
    return RECOIL_OK;
}

recoil_status recoil_batch_get_tuning(const recoil_batch *batch, recoil_tuning *t) {
    using namespace recoil;
    if (!batch || !t) return fail(RECOIL_ERR_INVALID_ARG, "batch_get_tuning: bad arguments");
    *t = batch->d.tuning;
    return RECOIL_OK;
}

recoil_status recoil_decode_batch(const recoil_batch *batch, void *d_ws, void *d_out, uint32_t *d_error, hipStream_t stream) {
    using namespace recoil;
    if (!batch || !d_ws || !d_out || !d_error) return fail(RECOIL_ERR_INVALID_ARG, "decode_batch: bad arguments");
    const BatchData &b = batch->d;
    hipError_t e = launch_classes(b, d_ws, d_out, d_error, stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode_batch: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

recoil_status recoil_decode_batch_noalloc(const recoil_batch *batch, const void *d_ws, void *d_out, uint32_t *d_error,
                                         hipStream_t stream) {
    using namespace recoil;
    if (!batch || !d_ws || !d_out || !d_error) return fail(RECOIL_ERR_INVALID_ARG, "decode_batch_noalloc: bad arguments");
    const BatchData &b = batch->d;
    // One queue head per table class in the library's static device array.
    static_assert(kBatchClasses * kStaticHeadStride <= kStaticScratchWords, "static queue heads do not fit");
    uint32_t classes = 0;
    for (uint32_t c = 0; c < kBatchClasses; ++c) classes += b.cls_count[c] ? 1u : 0u;
    if (classes * kStaticHeadStride > kStaticScratchWords)
        return fail(RECOIL_ERR_UNSUPPORTED, "decode_batch_noalloc: more table classes than static queue heads");
    uint32_t *heads = nullptr;
    hipError_t e = static_scratch(&heads);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode_batch_noalloc: ") + hipGetErrorString(e));
    // The workspace is only read: params_of's head pointer into it is replaced below.
    void *ws = const_cast<void *>(d_ws);
    for (uint32_t c = 0; c < kBatchClasses; ++c) {
        if (b.cls_count[c] == 0) continue;
        BatchParams bp = params_of(b, c, ws, d_out, d_error);
        bp.head = heads + c * kStaticHeadStride;
        e = launch_batch(bp, device_tuning(b.tuning), stream);
        if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode_batch_noalloc: ") + hipGetErrorString(e));
    }
    return RECOIL_OK;
}

recoil_status recoil_decode_batch_per_stream(const recoil_batch *batch, const void *d_ws, void *d_out,
                                             uint32_t *d_error, hipStream_t stream) {
    using namespace recoil;
    if (!batch || !d_ws || !d_out || !d_error) return fail(RECOIL_ERR_INVALID_ARG, "decode_batch_per_stream: bad arguments");
    const BatchData &b = batch->d;
    const char *ws = static_cast<const char *>(d_ws);
    char *out = static_cast<char *>(d_out);
    for (size_t i = 0; i < b.plans.size(); ++i) {
        const PlanData &pl = b.plans[i];
        const StreamDesc &d = b.descs[i];
        DecodeParams p{};
        p.words = reinterpret_cast<const uint16_t *>(ws + d.words_off);
        p.lut = ws + d.lut_off;
        p.meta = reinterpret_cast<const UnitMeta *>(ws + d.meta_off);
        p.lanes = reinterpret_cast<const uint32_t *>(ws + d.lanes_off);
        p.out = out + d.out_off;
        p.err = d_error;
        p.n_symbols = d.n_symbols;
        p.units = d.units;
        p.run = 1;
        p.runs = d.units;
        p.quant_bits = d.quant_bits;
        p.fill_symbol = d.fill_symbol;
        p.single_symbol = d.single_symbol;
        p.partitioned = d.partitioned;
        p.tables = 1;
        p.lut_bytes = (uint32_t)pl.lut.size();
        hipError_t e = launch_decode(p, pl.blob->lanes, pl.blob->symbol_bytes, pl.tuning, stream);
        if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("decode_batch_per_stream: ") + hipGetErrorString(e));
    }
    return RECOIL_OK;
}

recoil_status recoil_batch_graph_create(const recoil_batch *batch, void *d_ws, void *d_out, uint32_t *d_error,
                                        recoil_graph **out) {
    using namespace recoil;
    if (!batch || !out) return fail(RECOIL_ERR_INVALID_ARG, "batch_graph_create: bad arguments");
    *out = nullptr;
    auto *g = new (std::nothrow) recoil_graph();
    if (!g) return fail(RECOIL_ERR_INVALID_ARG, "batch_graph_create: out of memory");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const BatchData &b = batch->d;
        hipError_t le = launch_classes(b, d_ws, d_out, d_error, cs);
        e = hipStreamEndCapture(cs, &g->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return fail(RECOIL_ERR_HIP, std::string("batch_graph_create: ") + hipGetErrorString(e));
    }
    *out = g;
    return RECOIL_OK;
}

recoil_status recoil_graph_launch(recoil_graph *g, hipStream_t stream) {
    using namespace recoil;
    if (!g) return fail(RECOIL_ERR_INVALID_ARG, "graph_launch: NULL graph");
    hipError_t e = hipGraphLaunch(g->exec, stream);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("graph_launch: ") + hipGetErrorString(e));
    return RECOIL_OK;
}

void recoil_graph_free(recoil_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

recoil_status recoil_autotune(recoil_batch *batch, void *d_ws, void *d_out, uint32_t *d_error, hipStream_t stream,
                              uint32_t reps, recoil_tuning *best_out, float *best_ms) {
    using namespace recoil;
    if (!batch || !d_ws || !d_out || !d_error || reps == 0) return fail(RECOIL_ERR_INVALID_ARG, "autotune: bad arguments");
    BatchData &b = batch->d;
    // Cache key: device architecture plus the batch's shape.
    hipDeviceProp_t prop{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    uint64_t sym = 0, units = 0;
    uint32_t wide = 0;
    for (const PlanData &pl : b.plans) {
        sym += pl.blob->n_symbols;
        units += pl.blob->splits();
        wide += pl.blob->symbol_bytes == 2;
    }
    const std::string key = std::string(prop.gcnArchName) + "/" + std::to_string(b.plans.size()) + "/" +
                            std::to_string(sym) + "/" + std::to_string(units) + "/" + std::to_string(wide);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            recoil_status st = recoil_batch_set_tuning(batch, &it->second, d_ws, stream);
            if (st) return st;
            if (best_out) *best_out = it->second;
            if (best_ms) *best_ms = -1.0f;
            return RECOIL_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RECOIL_ERR_HIP, "autotune: event creation failed");
    recoil_tuning best{};
    float best_t = 1e30f;
    const uint32_t waves_opts[] = {8, 16}, k_opts[] = {4, 8}, p_opts[] = {1, 2, 4, 8}, r_opts[] = {1, 2, 4, 8};
    for (uint32_t w : waves_opts)
        for (uint32_t k : k_opts)
            for (uint32_t pp : p_opts)
            for (uint32_t ru : r_opts) {
                recoil_tuning t{w, k, pp, 0, ru};
                if (!shape_fits(b, t)) continue;
                if (recoil_batch_set_tuning(batch, &t, d_ws, stream)) continue;
                // Warm-up, then the median of `reps` timed launches.
                if (recoil_decode_batch(batch, d_ws, d_out, d_error, stream)) continue;
                std::vector<float> ts;
                for (uint32_t r = 0; r < reps; ++r) {
                    (void)hipEventRecord(e0, stream);
                    (void)recoil_decode_batch(batch, d_ws, d_out, d_error, stream);
                    (void)hipEventRecord(e1, stream);
                    (void)hipEventSynchronize(e1);
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ts.push_back(ms);
                }
                std::sort(ts.begin(), ts.end());
                const float med = ts[ts.size() / 2];
                if (med < best_t) { best_t = med; best = t; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_t >= 1e30f) return fail(RECOIL_ERR_HIP, "autotune: no configuration ran");
    recoil_status st = recoil_batch_set_tuning(batch, &best, d_ws, stream);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (best_out) *best_out = best;
    if (best_ms) *best_ms = best_t;
    return RECOIL_OK;
}

}  // extern "C"
