// Serving loop: resident content, per-request combine (Sec. 3.3), admission
// against a device budget and continuous batching of admitted requests onto the
// persistent batched decoder.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../device/batch.hpp"
#include "plan.hpp"
#include "recoil_batch.h"
#include "recoil_server.h"

namespace recoil {
namespace {

uint64_t clock_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over a byte range of the arena in 256-byte granules;
// neighbouring free blocks are merged on release.
class Budget {
  public:
    void reset(uint64_t lo, uint64_t hi) {
        free_.clear();
        cap_ = hi > lo ? hi - lo : 0;
        used_ = peak_ = 0;
        if (cap_) free_[lo] = cap_;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = ws_align(std::max<uint64_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            *off = o;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = ws_align(std::max<uint64_t>(bytes, 1));
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            free_.erase(next);
        }
        free_[off] = bytes;
    }
    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

  private:
    std::map<uint64_t, uint64_t> free_;   // offset -> bytes
    uint64_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Content {
    std::shared_ptr<const BlobData> blob;
    uint64_t words_off = 0, lut_off = 0;
    uint32_t lut_bytes = 0;
    bool single_symbol = false;
    uint32_t fill_symbol = 0;
};

struct Request {
    recoil_completion c{};
    Content content;
    uint32_t splits_asked = 0;
    uint64_t long_unit_bytes = 0;
    uint32_t single_max = 0;     // W = 32 requests of at most this many units decode one unit per wave
    PlanData plan;               // unit and lane records of the combined metadata
    uint64_t unit_bytes = 0;     // device bytes of the unit records (aligned)
    uint64_t meta_bytes = 0;     // unit + lane records (aligned)
    uint32_t pairs = 0;          // unit pairs (W = 32) or units (W = 64, or W = 32 one unit per wave)
    bool single = false;         // W = 32, one unit per wave
    uint32_t per_item = 0;       // pairs per work item in its launch
    uint32_t items = 0;          // work items in its launch
    bool is_long = false;        // many output bytes per decode unit (serial for long)
    bool completed = false;      // completion published (launcher thread only)
    std::atomic<int> ready{0};   // 1: planned; -1: failed (c.status says why)
};
using RequestPtr = std::shared_ptr<Request>;

// Control region of one launch slot (byte offsets): queue head, per-request
// error words, per-request outstanding item counts, stream descriptors, work items.
// The wide launch's queue head sits this many bytes after the first.
constexpr uint64_t kWideHeadOffset = 128;
struct CtrlLayout {
    uint64_t head = 0, err = 0, remaining = 0, descs = 0, items = 0, bytes = 0;
    CtrlLayout() = default;
    CtrlLayout(uint32_t max_batch, uint32_t max_items) {
        err = 256;
        remaining = err + ws_align((uint64_t)max_batch * 4);
        descs = remaining + ws_align((uint64_t)max_batch * 4);
        items = descs + ws_align((uint64_t)max_batch * sizeof(StreamDesc));
        bytes = ws_align(items + (uint64_t)max_items * sizeof(WorkItem));
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned char *staging = nullptr;   // pinned host memory
    size_t staging_cap = 0;
    uint32_t *done_host = nullptr;      // pinned, one completion word per request of the launch
    uint32_t *done_dev = nullptr;       // the same memory as the kernel addresses it
    uint64_t ctrl_off = 0;
    uint64_t meta_off = 0, meta_bytes = 0;
    std::vector<RequestPtr> reqs;
    bool busy = false;
    bool holds_long = false;            // the launch in flight carries a long request
};

}  // namespace
}  // namespace recoil

struct recoil_server {
    recoil_server_config cfg{};
    unsigned char *arena = nullptr;
    size_t arena_bytes = 0;
    int device = 0;
    uint64_t resident_end = 0, resident_used = 0, ctrl_bytes = 0;
    recoil::CtrlLayout ctrl{};
    recoil::BatchTuning tuning{};

    std::mutex mu;                                    // guards everything below up to the threads
    std::condition_variable cv_launcher, cv_done;
    std::vector<recoil::Content> contents;
    recoil::Budget budget;
    std::deque<recoil::RequestPtr> pending;
    std::deque<recoil_completion> done;
    std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> outputs;   // id -> (offset, bytes)
    bool stopping = false;
    uint64_t next_id = 1;
    uint64_t n_submitted = 0, n_completed = 0, n_rejected = 0, n_launches = 0, n_launched = 0, n_in_flight = 0;
    uint64_t decoded_bytes = 0;

    std::mutex prep_mu;
    std::condition_variable cv_prep;
    std::deque<recoil::RequestPtr> prep_q;
    bool prep_stop = false;

    std::vector<recoil::Slot> slots;                  // launcher thread only
    std::vector<std::thread> preppers;
    std::thread launcher;
};

namespace recoil {
namespace {

// Combine the content's split metadata down to the requested count: the
// per-unit records of the kept split points and the size of the metadata a
// client would receive (host work of one request, counted in its latency).
void prepare(Request &r) {
    const std::shared_ptr<const BlobData> &full = r.content.blob;
    const uint32_t M = full->splits();
    const uint32_t target = (r.splits_asked && r.splits_asked < M) ? r.splits_asked : M;
    uint64_t packed = 0;
    recoil_status st = build_units_combined(full, target, r.plan, &packed);
    if (st) {
        r.c.status = st;
        r.ready.store(-1, std::memory_order_release);
        return;
    }
    r.c.metadata_bytes = packed;
    const uint32_t Mc = (uint32_t)r.plan.meta.size();
    r.c.splits = Mc;
    r.c.out_bytes = full->n_symbols * full->symbol_bytes;
    r.unit_bytes = ws_align(Mc * sizeof(UnitMeta));
    r.meta_bytes = r.unit_bytes + ws_align((uint64_t)Mc * full->lanes * 4);
    r.single = full->lanes == 32 && Mc <= r.single_max;
    r.pairs = full->lanes == 32 && !r.single ? (Mc + 1) / 2 : Mc;
    r.is_long = r.c.out_bytes > r.long_unit_bytes * (uint64_t)Mc;
    r.ready.store(1, std::memory_order_release);
}

uint64_t items_of(const Request &r, uint32_t per_item) {
    const Content &ct = r.content;
    if (ct.blob->n_symbols == 0) return 0;
    if (ct.single_symbol) return 1;
    return (r.pairs + per_item - 1) / per_item;
}

void prep_loop(recoil_server *s) {
    for (;;) {
        RequestPtr r;
        {
            std::unique_lock<std::mutex> lk(s->prep_mu);
            s->cv_prep.wait(lk, [&] { return s->prep_stop || !s->prep_q.empty(); });
            if (s->prep_q.empty()) return;
            r = std::move(s->prep_q.front());
            s->prep_q.pop_front();
        }
        try {
            prepare(*r);
        } catch (...) {   // host memory exhausted while combining: the request fails, the server goes on
            r->c.status = RECOIL_ERR_OUT_OF_MEMORY;
            r->ready.store(-1, std::memory_order_release);
        }
        { std::lock_guard<std::mutex> lk(s->mu); }
        s->cv_launcher.notify_one();
    }
}

void complete_locked(recoil_server *s, Request &r) {
    s->done.push_back(r.c);
    ++s->n_completed;
    if (r.c.status == RECOIL_OK) s->decoded_bytes += r.c.out_bytes;
    else ++s->n_rejected;
    s->cv_done.notify_all();
}

void publish_locked(recoil_server *s, Request &r, uint64_t t) {
    r.c.t_done_ns = t;
    if (r.c.status == RECOIL_OK) s->outputs[r.c.request_id] = {r.c.out_offset, r.c.out_bytes};
    else s->budget.release(r.c.out_offset, r.c.out_bytes);
    r.completed = true;
    complete_locked(s, r);
}

// Publish requests whose completion word the kernel has set; when a launch's
// event has completed, publish the rest, free its unit records and the slot.
bool reap(recoil_server *s) {
    bool any = false;
    for (Slot &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        const bool finished = q != hipErrorNotReady;
        std::unique_lock<std::mutex> lk(s->mu, std::defer_lock);
        for (size_t i = 0; i < sl.reqs.size(); ++i) {
            Request &r = *sl.reqs[i];
            if (r.completed) continue;
            const uint32_t w = __atomic_load_n(sl.done_host + i, __ATOMIC_ACQUIRE);
            if (!(w & kHostDone) && !finished) continue;
            if (!lk.owns_lock()) lk.lock();
            if (w & kHostDone) r.c.device_error = w & ~kHostDone;
            else if (q != hipSuccess) r.c.status = RECOIL_ERR_HIP;
            publish_locked(s, r, clock_ns());
            any = true;
        }
        if (finished) {
            if (!lk.owns_lock()) lk.lock();
            s->budget.release(sl.meta_off, sl.meta_bytes);
            sl.reqs.clear();
            sl.busy = false;
            --s->n_in_flight;
            any = true;
        }
    }
    return any;
}

// Take, in queue order, the ready requests that fit one launch and the budget,
// passing over long ones when allow_long is false; called with s->mu held.
// Returns the admitted requests (may be empty) and removes them from the queue.
std::vector<RequestPtr> admit_locked(recoil_server *s, Slot &sl, bool idle, bool allow_long) {
    const uint32_t base_per_item = std::max(1u, s->cfg.tuning.waves * s->cfg.tuning.pairs_per_wave);
    std::vector<RequestPtr> take;
    uint64_t items = 0;
    for (size_t i = 0; i < s->pending.size() && take.size() < s->cfg.max_batch;) {
        RequestPtr r = s->pending[i];
        const int rd = r->ready.load(std::memory_order_acquire);
        if (rd == 0) break;
        if (rd < 0) {
            // Failed planning: complete at once.
            r->c.t_admit_ns = r->c.t_launch_ns = r->c.t_done_ns = clock_ns();
            s->pending.erase(s->pending.begin() + (ptrdiff_t)i);
            complete_locked(s, *r);
            continue;
        }
        ++i;
        if (r->is_long && !allow_long) continue;
        r->per_item = base_per_item;
        uint64_t n = items_of(*r, r->per_item);
        if (items + n > s->cfg.items_per_launch) {
            if (!take.empty()) break;
            r->per_item = (uint32_t)((r->pairs + s->cfg.items_per_launch - 1) / s->cfg.items_per_launch);
            n = items_of(*r, r->per_item);
        }
        items += n;
        take.push_back(r);
    }
    if (take.empty()) return take;
    // Outputs first, then one block for every admitted request's unit records;
    // drop requests from the back until both fit.
    size_t k = 0;
    for (; k < take.size(); ++k)
        if (!s->budget.alloc(take[k]->c.out_bytes, &take[k]->c.out_offset)) break;
    uint64_t meta = 0;
    for (size_t i = 0; i < k; ++i) meta += take[i]->meta_bytes;
    while (k > 0 && !s->budget.alloc(meta, &sl.meta_off)) {
        --k;
        s->budget.release(take[k]->c.out_offset, take[k]->c.out_bytes);
        meta -= take[k]->meta_bytes;
    }
    take.resize(k);
    if (k == 0) {
        // Nothing fits. If nothing else holds budget, this request never will.
        if (idle && s->budget.used() == 0) {
            RequestPtr r = s->pending.front();
            if (r->ready.load(std::memory_order_acquire) > 0 && (!r->is_long || allow_long)) {
                s->pending.pop_front();
                r->c.status = RECOIL_ERR_BUFFER_TOO_SMALL;
                r->c.t_admit_ns = r->c.t_launch_ns = r->c.t_done_ns = clock_ns();
                complete_locked(s, *r);
            }
        }
        return take;
    }
    // A launch whose pairs would not fill its resident workgroups (the usual case
    // below full load) cuts its requests into smaller items, about one per
    // workgroup, so that each request spreads over many CUs instead of a few:
    // a request's latency is then its own decode time.
    {
        uint64_t pairs = 0;
        uint32_t lut = 16;
        for (const RequestPtr &r : take) {
            pairs += r->pairs;
            lut = std::max(lut, r->content.lut_bytes);
        }
        const uint64_t wgs = (uint64_t)std::max(batch_blocks_per_cu(s->tuning, lut), 0) * (uint64_t)device_cus();
        if (wgs > 0 && pairs < wgs * base_per_item) {
            const uint32_t fine = (uint32_t)std::max<uint64_t>(1, (pairs + wgs - 1) / wgs);
            uint64_t n = 0;
            for (const RequestPtr &r : take) n += items_of(*r, std::min(r->per_item, fine));
            if (n <= s->cfg.items_per_launch)
                for (RequestPtr &r : take) r->per_item = std::min(r->per_item, fine);
        }
    }
    sl.meta_bytes = meta;
    sl.holds_long = false;
    const uint64_t t = clock_ns();
    for (RequestPtr &r : take) {
        r->c.t_admit_ns = t;
        sl.holds_long = sl.holds_long || r->is_long;
    }
    // Remove the admitted requests from the queue (they are in queue order).
    size_t j = 0;
    auto keep = std::remove_if(s->pending.begin(), s->pending.end(), [&](const RequestPtr &r) {
        if (j < take.size() && r == take[j]) { ++j; return true; }
        return false;
    });
    s->pending.erase(keep, s->pending.end());
    return take;
}

// Stage descriptors, items and unit records of an admitted set and enqueue
// [copies; queue reset + persistent decode; error word back; event] on the slot.
hipError_t launch_slot(recoil_server *s, Slot &sl) {
    const uint32_t k = (uint32_t)sl.reqs.size();
    const CtrlLayout &L = s->ctrl;
    uint64_t n_items = 0;
    for (RequestPtr &r : sl.reqs) {
        r->items = (uint32_t)items_of(*r, r->per_item);
        n_items += r->items;
    }
    const uint64_t ctrl_used = L.items + n_items * sizeof(WorkItem);
    const uint64_t need = s->ctrl_bytes + sl.meta_bytes;
    if (need > sl.staging_cap) {
        if (sl.staging) (void)hipHostFree(sl.staging);
        sl.staging = nullptr;
        sl.staging_cap = 0;
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&sl.staging), need, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        sl.staging_cap = need;
    }
    unsigned char *ctrl = sl.staging;
    unsigned char *meta = sl.staging + s->ctrl_bytes;
    std::memset(ctrl, 0, L.descs);       // queue head and error words start at zero
    uint32_t *remaining = reinterpret_cast<uint32_t *>(ctrl + L.remaining);
    for (uint32_t i = 0; i < k; ++i) remaining[i] = sl.reqs[i]->items;
    std::memset(sl.done_host, 0, (size_t)k * 4);
    StreamDesc *descs = reinterpret_cast<StreamDesc *>(ctrl + L.descs);
    WorkItem *items = reinterpret_cast<WorkItem *>(ctrl + L.items);
    uint32_t lut_bytes[2] = {16, 16};     // largest table of the one-level and of the wide requests
    uint64_t moff = 0;
    for (uint32_t i = 0; i < k; ++i) {
        const Request &r = *sl.reqs[i];
        const Content &ct = r.content;
        const BlobData &b = *ct.blob;
        StreamDesc &d = descs[i];
        std::memset(&d, 0, sizeof(d));
        d.words_off = ct.words_off;
        d.lut_off = ct.lut_off;
        d.meta_off = sl.meta_off + moff;
        d.lanes_off = sl.meta_off + moff + r.unit_bytes;
        d.out_off = r.c.out_offset;
        d.n_symbols = b.n_symbols;
        d.units = r.c.splits;
        d.quant_bits = (uint8_t)b.quant_bits;
        d.symbol_bytes = (uint8_t)b.symbol_bytes;
        d.lanes = (uint8_t)b.lanes;
        d.single_symbol = ct.single_symbol ? 1 : 0;
        d.fill_symbol = ct.fill_symbol;
        d.lut_chunks = (uint16_t)(ct.lut_bytes / 16);
        std::memcpy(meta + moff, r.plan.meta.data(), r.plan.meta.size() * sizeof(UnitMeta));
        std::memcpy(meta + moff + r.unit_bytes, r.plan.lanes.data(), r.plan.lanes.size() * 4);
        moff += r.meta_bytes;
        lut_bytes[b.quant_bits > 12] = std::max(lut_bytes[b.quant_bits > 12], ct.lut_bytes);
    }
    // Requests with one-level tables first, then those with two-level tables (13 <= n
    // <= 16, a kernel of their own); in each, the largest request first, so the
    // longest work starts first.
    auto wide = [&](uint32_t i) { return sl.reqs[i]->content.blob->quant_bits > 12; };
    std::vector<uint32_t> order(k);
    for (uint32_t i = 0; i < k; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (wide(a) != wide(b)) return !wide(a);
        return sl.reqs[a]->c.out_bytes > sl.reqs[b]->c.out_bytes;
    });
    uint64_t it = 0, n_plain = 0;
    bool seen_wide = false;
    for (uint32_t i : order) {
        if (wide(i) && !seen_wide) {
            n_plain = it;
            seen_wide = true;
        }
        const Request &r = *sl.reqs[i];
        if (r.items == 0) continue;
        if (r.content.single_symbol) { items[it++] = WorkItem{i, 0, 1, 0}; continue; }
        for (uint64_t f = 0; f < r.pairs; f += r.per_item)
            items[it++] = WorkItem{i, (uint32_t)f, (uint32_t)std::min<uint64_t>(r.per_item, r.pairs - f),
                                   r.single ? kItemSingle : 0u};
    }
    if (!seen_wide) n_plain = it;
    unsigned char *a = s->arena;
    hipError_t e = hipMemcpyAsync(a + sl.ctrl_off, ctrl, ctrl_used, hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess && sl.meta_bytes)
        e = hipMemcpyAsync(a + sl.meta_off, meta, sl.meta_bytes, hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return e;
    BatchParams bp{};
    bp.ws = a;
    bp.out = a;
    bp.streams = reinterpret_cast<const StreamDesc *>(a + sl.ctrl_off + L.descs);
    bp.items = reinterpret_cast<const WorkItem *>(a + sl.ctrl_off + L.items);
    bp.head = reinterpret_cast<uint32_t *>(a + sl.ctrl_off + L.head);
    bp.err = reinterpret_cast<uint32_t *>(a + sl.ctrl_off + L.err);
    bp.err_stride = 1;
    bp.remaining = reinterpret_cast<uint32_t *>(a + sl.ctrl_off + L.remaining);
    bp.host_done = sl.done_dev;
    const uint64_t t = clock_ns();
    for (RequestPtr &r : sl.reqs) r->c.t_launch_ns = t;
    // One persistent launch for the one-level tables' items, then one for the wide
    // tables' items with its own queue head (128 bytes on).
    bp.n_items = (uint32_t)n_plain;
    bp.lut_bytes = lut_bytes[0];
    e = launch_batch(bp, s->tuning, sl.stream);
    if (e == hipSuccess && n_items > n_plain) {
        bp.items += n_plain;
        bp.head = reinterpret_cast<uint32_t *>(a + sl.ctrl_off + L.head + kWideHeadOffset);
        bp.n_items = (uint32_t)(n_items - n_plain);
        bp.lut_bytes = lut_bytes[1];
        bp.wide = 1;
        e = launch_batch(bp, s->tuning, sl.stream);
    }
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    return e;
}

void launcher_loop(recoil_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        reap(s);
        std::unique_lock<std::mutex> lk(s->mu);
        bool busy = false;
        uint32_t long_in_flight = 0;
        Slot *free_slot = nullptr;
        for (Slot &sl : s->slots) {
            if (sl.busy) {
                busy = true;
                long_in_flight += sl.holds_long;
            } else if (!free_slot) {
                free_slot = &sl;
            }
        }
        if (s->stopping) {
            if (!busy) break;
            lk.unlock();
            std::this_thread::yield();
            continue;
        }
        if (free_slot) {
            std::vector<RequestPtr> take = admit_locked(s, *free_slot, !busy, long_in_flight < s->cfg.long_streams);
            if (!take.empty()) {
                free_slot->reqs = std::move(take);
                free_slot->busy = true;
                ++s->n_launches;
                s->n_launched += free_slot->reqs.size();
                ++s->n_in_flight;
                lk.unlock();
                hipError_t e;
                try {
                    e = launch_slot(s, *free_slot);
                } catch (...) {   // host memory exhausted while staging the set
                    e = hipErrorOutOfMemory;
                }
                if (e != hipSuccess) {
                    // Nothing (or only part) was enqueued: fail the set and wait for the stream to drain.
                    (void)hipStreamSynchronize(free_slot->stream);
                    std::lock_guard<std::mutex> lk2(s->mu);
                    s->budget.release(free_slot->meta_off, free_slot->meta_bytes);
                    for (RequestPtr &r : free_slot->reqs) {
                        r->c.status = RECOIL_ERR_HIP;
                        r->c.t_done_ns = clock_ns();
                        s->budget.release(r->c.out_offset, r->c.out_bytes);
                        complete_locked(s, *r);
                    }
                    free_slot->reqs.clear();
                    free_slot->busy = false;
                    --s->n_in_flight;
                }
                continue;
            }
        }
        // Launches in flight: poll their events often; idle: sleep until woken.
        if (busy) s->cv_launcher.wait_for(lk, std::chrono::microseconds(20));
        else s->cv_launcher.wait_for(lk, std::chrono::milliseconds(5));
    }
}

void destroy_slots(recoil_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.done_host) (void)hipHostFree(sl.done_host);
        sl = Slot{};
    }
}

}  // namespace
}  // namespace recoil

extern "C" {

uint64_t recoil_server_now_ns(void) { return recoil::clock_ns(); }

recoil_status recoil_server_create(const recoil_server_config *cfg, void *d_arena, size_t arena_bytes,
                                   recoil_server **out) {
    return recoil::guarded("server_create", [&]() -> recoil_status {
    using namespace recoil;
    if (!cfg || !d_arena || !out) return fail(RECOIL_ERR_INVALID_ARG, "server_create: bad arguments");
    *out = nullptr;
    if (cfg->hip_streams < 1 || cfg->hip_streams > 8 || cfg->max_batch < 1 || cfg->max_batch > 4096 ||
        cfg->prep_threads < 1 || cfg->prep_threads > 64 || cfg->items_per_launch < 1024 ||
        cfg->items_per_launch > (1u << 22))
        return fail(RECOIL_ERR_INVALID_ARG, "server_create: configuration out of range");
    const recoil_tuning &t = cfg->tuning;
    if (!((t.waves == 8 || t.waves == 16) && (t.chunk_groups == 4 || t.chunk_groups == 8) && t.pairs_per_wave >= 1 &&
          t.pairs_per_wave <= 64))
        return fail(RECOIL_ERR_INVALID_ARG, "server_create: unsupported tuning");
    if (reinterpret_cast<uintptr_t>(d_arena) % kWsAlign)
        return fail(RECOIL_ERR_ALIGNMENT, "server_create: arena not 256-byte aligned");
    const uint64_t resident_end = ws_align(cfg->resident_bytes);
    const CtrlLayout layout(cfg->max_batch, cfg->items_per_launch);
    const uint64_t ctrl = layout.bytes;
    const uint64_t ctrl_total = ctrl * cfg->hip_streams;
    if (resident_end + ctrl_total >= arena_bytes)
        return fail(RECOIL_ERR_INVALID_ARG, "server_create: arena too small for the resident and control regions");
    auto *s = new (std::nothrow) recoil_server();
    if (!s) return fail(RECOIL_ERR_INVALID_ARG, "server_create: out of memory");
    s->cfg = *cfg;
    if (s->cfg.long_unit_bytes == 0) s->cfg.long_unit_bytes = 131072;
    if (s->cfg.long_streams == 0) s->cfg.long_streams = std::max(1u, cfg->hip_streams / 2);
    s->arena = static_cast<unsigned char *>(d_arena);
    s->arena_bytes = arena_bytes;
    s->resident_end = resident_end;
    s->ctrl_bytes = ctrl;
    s->ctrl = layout;
    s->tuning = BatchTuning{t.waves, t.chunk_groups, t.blocks_per_cu};
    s->budget.reset(resident_end + ctrl_total, arena_bytes / kWsAlign * kWsAlign);
    hipError_t e = hipGetDevice(&s->device);
    s->slots.resize(cfg->hip_streams);
    for (uint32_t i = 0; e == hipSuccess && i < cfg->hip_streams; ++i) {
        Slot &sl = s->slots[i];
        sl.ctrl_off = resident_end + (uint64_t)i * ctrl;
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&sl.done_host), (size_t)cfg->max_batch * 4, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.done_dev), sl.done_host, 0);
    }
    if (e != hipSuccess) {
        destroy_slots(s);
        delete s;
        return fail(RECOIL_ERR_HIP, std::string("server_create: ") + hipGetErrorString(e));
    }
    try {
        for (uint32_t i = 0; i < cfg->prep_threads; ++i) s->preppers.emplace_back(prep_loop, s);
        s->launcher = std::thread(launcher_loop, s);
    } catch (...) {
        // A thread could not be started: stop the ones that were, then report.
        {
            std::lock_guard<std::mutex> lk(s->prep_mu);
            s->prep_stop = true;
        }
        s->cv_prep.notify_all();
        for (std::thread &t : s->preppers) t.join();
        destroy_slots(s);
        delete s;
        throw;
    }
    *out = s;
    return RECOIL_OK;
    });
}

recoil_status recoil_server_add_content(recoil_server *s, const recoil_blob *blob, uint32_t *content_id) {
    return recoil::guarded("server_add_content", [&]() -> recoil_status {
    using namespace recoil;
    if (!s || !blob || !content_id) return fail(RECOIL_ERR_INVALID_ARG, "server_add_content: bad arguments");
    const std::shared_ptr<const BlobData> &bp = blob->data;
    if (bp->partitioned())   // requests ask for a unit count, which a partitioned stream cannot give
        return fail(RECOIL_ERR_UNSUPPORTED, "server_add_content: partitioned streams cannot be combined per request");
    if (bp->adaptive) return fail(RECOIL_ERR_UNSUPPORTED, "server_add_content: adaptive streams are decoded alone");
    PlanData probe;
    recoil_status st = build_units(bp, probe);   // checks the GPU decoder's limits
    if (st) return st;
    build_table(*bp, probe);
    Content ct;
    ct.blob = bp;
    ct.lut_bytes = (uint32_t)probe.lut.size();
    ct.single_symbol = probe.single_symbol;
    ct.fill_symbol = probe.fill_symbol;
    if (batch_blocks_per_cu(s->tuning, ct.lut_bytes, bp->quant_bits > 12) < 1)
        return fail(RECOIL_ERR_UNSUPPORTED, "server_add_content: decode table does not fit the launch shape");
    const uint64_t wbytes = words_section_bytes(bp->n_words());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return fail(RECOIL_ERR_INVALID_ARG, "server_add_content: server is shutting down");
        if (s->resident_used + wbytes + ws_align(ct.lut_bytes) > s->resident_end)
            return fail(RECOIL_ERR_BUFFER_TOO_SMALL, "server_add_content: resident region full");
        ct.words_off = s->resident_used;
        ct.lut_off = s->resident_used + wbytes;
        s->resident_used += wbytes + ws_align(ct.lut_bytes);
    }
    hipError_t e = hipSuccess;
    if (bp->n_words()) e = stage_h2d(s->arena + ct.words_off, bp->words(), 2 * bp->n_words(), nullptr);
    if (e == hipSuccess) e = stage_h2d(s->arena + ct.lut_off, probe.lut.data(), probe.lut.size(), nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return fail(RECOIL_ERR_HIP, std::string("server_add_content: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(s->mu);
    *content_id = (uint32_t)s->contents.size();
    s->contents.push_back(std::move(ct));
    return RECOIL_OK;
    });
}

recoil_status recoil_server_submit(recoil_server *s, uint32_t content, uint32_t splits, uint64_t tag,
                                   uint64_t arrival_ns, uint64_t *request_id) {
    return recoil::guarded("server_submit", [&]() -> recoil_status {
    using namespace recoil;
    if (!s) return fail(RECOIL_ERR_INVALID_ARG, "server_submit: NULL server");
    auto r = std::make_shared<Request>();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return fail(RECOIL_ERR_INVALID_ARG, "server_submit: server is shutting down");
        if (content >= s->contents.size()) return fail(RECOIL_ERR_INVALID_ARG, "server_submit: unknown content");
        r->content = s->contents[content];
        r->splits_asked = splits;
        r->long_unit_bytes = s->cfg.long_unit_bytes;
        r->single_max = s->cfg.tuning.waves;
        r->c.request_id = s->next_id++;
        r->c.tag = tag;
        r->c.content = content;
        r->c.status = RECOIL_OK;
        r->c.t_arrival_ns = arrival_ns ? arrival_ns : clock_ns();
        s->pending.push_back(r);
        ++s->n_submitted;
        if (request_id) *request_id = r->c.request_id;
    }
    {
        std::lock_guard<std::mutex> lk(s->prep_mu);
        s->prep_q.push_back(r);
    }
    s->cv_prep.notify_one();
    return RECOIL_OK;
    });
}

uint32_t recoil_server_poll(recoil_server *s, recoil_completion *done, uint32_t cap, uint32_t timeout_us) {
    if (!s || !done || cap == 0) return 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_us)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
    uint32_t n = 0;
    while (n < cap && !s->done.empty()) {
        done[n++] = s->done.front();
        s->done.pop_front();
    }
    return n;
}

recoil_status recoil_server_release(recoil_server *s, uint64_t request_id) {
    using namespace recoil;
    if (!s) return fail(RECOIL_ERR_INVALID_ARG, "server_release: NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->outputs.find(request_id);
        if (it == s->outputs.end()) return fail(RECOIL_ERR_INVALID_ARG, "server_release: unknown or released request");
        s->budget.release(it->second.first, it->second.second);
        s->outputs.erase(it);
    }
    s->cv_launcher.notify_one();
    return RECOIL_OK;
}

recoil_status recoil_server_get_stats(const recoil_server *cs, recoil_server_stats *st) {
    using namespace recoil;
    if (!cs || !st) return fail(RECOIL_ERR_INVALID_ARG, "server_get_stats: bad arguments");
    auto *s = const_cast<recoil_server *>(cs);
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->n_submitted;
    st->completed = s->n_completed;
    st->rejected = s->n_rejected;
    st->launches = s->n_launches;
    st->requests_launched = s->n_launched;
    st->pending = s->pending.size();
    st->in_flight = s->n_in_flight;
    st->budget_bytes = s->budget.capacity();
    st->budget_used = s->budget.used();
    st->budget_peak = s->budget.peak();
    st->resident_used = s->resident_used;
    st->decoded_bytes = s->decoded_bytes;
    return RECOIL_OK;
}

void recoil_server_destroy(recoil_server *s) {
    using namespace recoil;
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->pending.clear();
    }
    s->cv_launcher.notify_all();
    if (s->launcher.joinable()) s->launcher.join();
    {
        std::lock_guard<std::mutex> lk(s->prep_mu);
        s->prep_stop = true;
        s->prep_q.clear();
    }
    s->cv_prep.notify_all();
    for (std::thread &t : s->preppers) t.join();
    destroy_slots(s);
    delete s;
}

}  // extern "C"
