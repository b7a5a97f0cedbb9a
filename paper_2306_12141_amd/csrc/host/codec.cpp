// librecoil host codec: table quantisation, interleaved rANS encoding with
// streaming split selection, container packing/validation and split combining.
//
// Method references (Lin et al., ICPP 2023): Eq. 1 and Eq. 3 (encode step and
// renormalisation), Sec. 2.2 (interleaving), Sec. 4.1 (backward scan), Def. 4.1
// (split heuristic), Sec. 3.3 (combining), Sec. 4.3 (metadata storage).
#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <queue>
#include <thread>
#include <utility>

#include "blob.hpp"

namespace recoil {

namespace {
thread_local std::string g_last_error;

inline uint64_t cdiv(uint64_t a, uint64_t b) { return b ? (a + b - 1) / b : 0; }

inline uint32_t bitlen(uint64_t v) { return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u; }

// MSB-first bit sink with a 64-bit accumulator.
class BitSink {
public:
    explicit BitSink(std::vector<uint8_t> &out) : out_(out) {}
    void put(uint64_t v, uint32_t w) {
        while (w) {
            uint32_t take = std::min<uint32_t>(w, 32);
            uint64_t part = (v >> (w - take)) & ((1ull << take) - 1);
            acc_ = (acc_ << take) | part;
            n_ += take;
            w -= take;
            while (n_ >= 8) {
                n_ -= 8;
                out_.push_back((uint8_t)(acc_ >> n_));
            }
            acc_ &= (n_ ? ((1ull << n_) - 1) : 0);
        }
    }
    void flush() {
        if (n_) out_.push_back((uint8_t)(acc_ << (8 - n_)));
        n_ = 0;
        acc_ = 0;
    }
    uint64_t bit_pos() const { return 8ull * out_.size() + n_; }

private:
    std::vector<uint8_t> &out_;
    uint64_t acc_ = 0;
    uint32_t n_ = 0;
};

class BitSource {
public:
    BitSource(const uint8_t *p, uint64_t nbytes) : p_(p), nbits_(nbytes * 8) {}
    // Returns false on overrun.
    bool get(uint32_t w, uint64_t &v) {
        if (w > nbits_ - pos_ || pos_ > nbits_) return false;
        v = 0;
        while (w) {
            uint64_t byte = pos_ >> 3;
            uint32_t off = (uint32_t)(pos_ & 7);
            uint32_t avail = 8 - off;
            uint32_t take = std::min(avail, w);
            uint32_t bits = ((uint32_t)p_[byte] >> (avail - take)) & ((1u << take) - 1);
            v = (v << take) | bits;
            pos_ += take;
            w -= take;
        }
        return true;
    }
    uint64_t pos() const { return pos_; }

private:
    const uint8_t *p_;
    uint64_t nbits_;
    uint64_t pos_ = 0;
};

template <class Get>
bool put_series(BitSink &s, uint64_t count, uint32_t field, bool is_signed, Get get) {
    uint64_t maxmag = 0;
    for (uint64_t k = 0; k < count; ++k) {
        int64_t v = get(k);
        if (!is_signed && v < 0) return false;
        uint64_t m = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        maxmag = std::max(maxmag, m);
    }
    uint32_t width = std::max<uint32_t>(1, bitlen(maxmag));
    if (width - 1 >= (1u << field)) return false;
    s.put(width - 1, field);
    for (uint64_t k = 0; k < count; ++k) {
        int64_t v = get(k);
        uint64_t m = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        if (is_signed) {
            s.put((v < 0) ? 1 : 0, 1);
        }
        s.put(m, width);
    }
    return true;
}

bool get_series(BitSource &s, uint64_t count, uint32_t field, bool is_signed, std::vector<int64_t> &out) {
    uint64_t w1;
    if (!s.get(field, w1)) return false;
    uint32_t width = (uint32_t)w1 + 1;
    if (width > 63) return false;
    out.resize(count);
    for (uint64_t k = 0; k < count; ++k) {
        uint64_t sign = 0, mag;
        if (is_signed && !s.get(1, sign)) return false;
        if (!s.get(width, mag)) return false;
        out[k] = sign ? -(int64_t)mag : (int64_t)mag;
    }
    return true;
}

void put_u(std::vector<uint8_t> &v, uint64_t x, int n) {
    for (int k = 0; k < n; ++k) v.push_back((uint8_t)(x >> (8 * k)));
}
uint64_t get_u(const uint8_t *p, int n) {
    uint64_t x = 0;
    for (int k = 0; k < n; ++k) x |= (uint64_t)p[k] << (8 * k);
    return x;
}

// --------------------------------------------------------------------------
// Streaming split selection.
//
// The encoder reports every renormalisation event (word position, symbol index
// of the lane's previous symbol, post-shift state). A word is a candidate split
// point once every lane has a non-negative event at or before it; Imin is the
// oldest of those lanes' latest events (tracked with a recency list), Imax the
// event of the word itself. The greedy choice of Def. 4.1 is evaluated while
// encoding: for split k the target T is recomputed from the remaining symbols,
// the window closes at the first candidate with t > 2T + t_s, ties go to the
// earliest word. Only the candidates and events since the last chosen split
// are kept; the chosen split's per-lane records come from a backward scan over
// those events, falling back to the previous split's records.
// --------------------------------------------------------------------------
class SplitChooser {
public:
    SplitChooser(BlobData &b, uint32_t threads) : b_(b), W_(b.lanes), M_(threads) {
        last_.assign(W_, -1);
        prv_.assign(W_, -1);
        nxt_.assign(W_, -1);
        snap_idx_.assign(W_, -1);
        snap_state_.assign(W_, 0);
        scan_seen_.assign(W_, 0);
        retarget();
    }

    bool done() const { return k_ >= M_; }

    void event(uint64_t pos, int64_t idx, uint32_t state) {
        if (done()) return;
        ev_.push_back({pos, idx, (uint16_t)state});
        if (idx < 0) return;
        const uint32_t lane = (uint32_t)((uint64_t)idx % W_);
        if (last_[lane] < 0) {
            ++valid_;
            append(lane);
        } else {
            unlink(lane);
            append(lane);
        }
        last_[lane] = idx;
        if (valid_ < W_) return;
        const int64_t imin = last_[head_];
        if ((uint64_t)(idx / W_ - imin / W_) > kMaxGroupDiff) return;
        cand_.push_back({pos, idx, imin});
        run();
    }

    void finish() {
        while (!done() && have_best_) {
            choose();
            run();
        }
    }

private:
    struct Ev { uint64_t pos; int64_t idx; uint16_t state; };
    struct Cand { uint64_t pos; int64_t imax, imin; };

    void append(uint32_t lane) {
        prv_[lane] = tail_;
        nxt_[lane] = -1;
        if (tail_ >= 0) nxt_[tail_] = (int32_t)lane; else head_ = (int32_t)lane;
        tail_ = (int32_t)lane;
    }
    void unlink(uint32_t lane) {
        int32_t p = prv_[lane], n = nxt_[lane];
        if (p >= 0) nxt_[p] = n; else head_ = n;
        if (n >= 0) prv_[n] = p; else tail_ = p;
    }

    void retarget() {
        if (done()) return;
        int64_t remaining = (int64_t)b_.n_symbols - prev_max_ - 1;
        if (remaining < 0) remaining = 0;
        T_ = (int64_t)cdiv((uint64_t)remaining, M_ - k_ + 1);
    }

    void run() {
        while (!done() && head_c_ < cand_.size()) {
            const Cand &c = cand_[head_c_];
            const int64_t t = c.imax - prev_max_;
            const int64_t ts = c.imax - c.imin + 1;
            const bool beyond = t > 2 * T_ + ts;
            if (have_best_ && beyond) { choose(); continue; }
            const int64_t h = std::llabs(t - T_) + std::llabs(t - ts - T_);
            if (!have_best_ || h < best_h_) { have_best_ = true; best_ = head_c_; best_h_ = h; }
            if (beyond) { choose(); continue; }
            ++head_c_;
        }
    }

    void choose() {
        const Cand c = cand_[best_];
        // Backward scan from the chosen word over the events kept since the last split.
        std::fill(scan_seen_.begin(), scan_seen_.end(), 0);
        size_t e = ev_.size();
        while (e > 0 && ev_[e - 1].pos > c.pos) --e;
        uint32_t seen = 0;
        const size_t base = b_.sp_state.size();
        b_.sp_state.resize(base + W_);
        b_.sp_gdiff.resize(base + W_);
        std::vector<int64_t> idx(W_, -1);
        for (size_t q = e; q > 0 && seen < W_; --q) {
            const Ev &ev = ev_[q - 1];
            if (ev.idx < 0) continue;
            uint32_t lane = (uint32_t)((uint64_t)ev.idx % W_);
            if (scan_seen_[lane]) continue;
            scan_seen_[lane] = 1;
            ++seen;
            idx[lane] = ev.idx;
            b_.sp_state[base + lane] = ev.state;
        }
        for (uint32_t j = 0; j < W_; ++j) {
            if (!scan_seen_[j]) { idx[j] = snap_idx_[j]; b_.sp_state[base + j] = snap_state_[j]; }
            snap_idx_[j] = idx[j];
            snap_state_[j] = b_.sp_state[base + j];
        }
        const uint64_t anchor = (uint64_t)c.imax / W_;
        for (uint32_t j = 0; j < W_; ++j)
            b_.sp_gdiff[base + j] = (uint16_t)(anchor - (uint64_t)idx[j] / W_);
        b_.sp_next.push_back(c.pos + 1);
        b_.sp_anchor.push_back(anchor);
        // Drop what the next split can no longer need.
        ev_.erase(ev_.begin(), ev_.begin() + (ptrdiff_t)e);
        cand_.erase(cand_.begin(), cand_.begin() + (ptrdiff_t)best_ + 1);
        head_c_ = 0;
        have_best_ = false;
        prev_max_ = c.imax;
        ++k_;
        retarget();
        if (done()) { ev_.clear(); cand_.clear(); }
    }

    BlobData &b_;
    const uint32_t W_;
    const uint32_t M_;
    uint32_t k_ = 1;
    int64_t prev_max_ = -1;
    int64_t T_ = 0;
    bool have_best_ = false;
    size_t best_ = 0;
    int64_t best_h_ = 0;
    size_t head_c_ = 0;
    uint32_t valid_ = 0;
    int32_t head_ = -1, tail_ = -1;
    std::vector<int64_t> last_;
    std::vector<int32_t> prv_, nxt_;
    std::vector<int64_t> snap_idx_;
    std::vector<uint16_t> snap_state_;
    std::vector<uint8_t> scan_seen_;
    std::vector<Ev> ev_;
    std::vector<Cand> cand_;
};

// --------------------------------------------------------------------------
// Parallel split writer.
//
// The same choice as SplitChooser, in three passes over a log the encoder keeps
// (per word: the index of the symbol being encoded when it was emitted, so the
// event's own index is that minus W, and the post-shift state):
//  1. per chunk of words, each lane's latest event inside the chunk (threads);
//     a prefix over the chunks gives each chunk the lanes' latest events before it;
//  2. per chunk, Imin at every word (oldest of the lanes' latest events, a
//     recency list started from the carried-in events) and the streaming
//     candidate test (threads);
//  3. the greedy choice of Def. 4.1, split by split. Imax grows strictly and Imin
//     never falls from word to word, so with c = Imax_{k-1} + T the score
//     H = |t - T| + |t - t_s - T| = |Imax - c| + |Imin - 1 - c| falls strictly
//     while Imax < c, equals t_s while Imax >= c >= Imin - 1, and rises strictly
//     once Imin - 1 > c; the window ends at the first candidate with
//     Imin > c + T + 1 (t > 2T + t_s). Binary searches find those boundaries and
//     only the last falling candidate, the level ones and the first rising one
//     are scored, in word order with ties to the earlier word, as the streaming
//     chooser scores the whole window. The chosen words' backward scans follow.
// --------------------------------------------------------------------------
std::atomic<uint32_t> g_split_threads{0};   // 0: automatic, 1: streaming chooser, >= 2: this many threads

constexpr uint64_t kParallelSplitMinSymbols = 1ull << 24;
// Per-word key of pass 2: Imin + 1 in bits 0..30 (0 before every lane has an event),
// bit 31 set when the word is no candidate.
constexpr uint32_t kNotCandidate = 0x80000000u;

uint32_t split_writer_threads(uint64_t n_symbols) {
    const uint32_t t = g_split_threads.load(std::memory_order_relaxed);
    if (t) return t;
    if (n_symbols < kParallelSplitMinSymbols) return 1;
    return std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
}

struct EventLog {
    std::vector<uint32_t> sym;     // per word: index of the symbol being encoded
    std::vector<uint16_t> state;   // per word: post-shift state
};

void choose_splits_parallel(BlobData &b, const EventLog &log, uint32_t M, uint32_t threads) {
    const uint32_t W = b.lanes;
    const uint64_t B = log.sym.size();
    const uint32_t chunks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(threads, B / 4096 + 1));
    auto chunk_lo = [&](uint32_t c) { return B * c / chunks; };
    // Chunk c on a thread of its own (chunk 0 on the caller's). A thread that cannot
    // be started leaves its chunks to the caller; a failure inside a chunk is
    // reported once every thread has been joined.
    auto run = [&](auto &&fn) {
        std::atomic<bool> failed{false};
        auto body = [&](uint32_t c) {
            try { fn(c); } catch (...) { failed = true; }
        };
        std::vector<std::thread> ts;
        uint32_t c = 1;
        try {
            for (; c < chunks; ++c) ts.emplace_back(body, c);
        } catch (...) {
        }
        for (uint32_t r = c; r < chunks; ++r) body(r);
        body(0u);
        for (std::thread &t : ts) t.join();
        if (failed) throw std::bad_alloc();
    };
    // Pass 1: each lane's latest event inside each chunk.
    std::vector<int64_t> last((size_t)chunks * W, -1);
    run([&](uint32_t c) {
        int64_t *l = &last[(size_t)c * W];
        for (uint64_t w = chunk_lo(c); w < chunk_lo(c + 1); ++w) {
            const int64_t idx = (int64_t)log.sym[w] - (int64_t)W;
            if (idx >= 0) l[(uint64_t)idx % W] = idx;
        }
    });
    std::vector<int64_t> carry((size_t)chunks * W, -1);
    for (uint32_t c = 1; c < chunks; ++c)
        for (uint32_t j = 0; j < W; ++j) {
            const int64_t v = last[(size_t)(c - 1) * W + j];
            carry[(size_t)c * W + j] = v >= 0 ? v : carry[(size_t)(c - 1) * W + j];
        }
    // Pass 2: Imin at every word and the candidate test.
    std::vector<uint32_t> key(B, 0);
    run([&](uint32_t c) {
        std::vector<int64_t> lst(carry.begin() + (size_t)c * W, carry.begin() + (size_t)(c + 1) * W);
        std::vector<int32_t> prv(W, -1), nxt(W, -1), order;
        int32_t head = -1, tail = -1;
        uint32_t valid = 0;
        for (uint32_t j = 0; j < W; ++j) if (lst[j] >= 0) order.push_back((int32_t)j);
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t z) { return lst[a] < lst[z]; });
        auto append = [&](int32_t j) {
            prv[j] = tail; nxt[j] = -1;
            if (tail >= 0) nxt[tail] = j; else head = j;
            tail = j;
        };
        auto unlink = [&](int32_t j) {
            if (prv[j] >= 0) nxt[prv[j]] = nxt[j]; else head = nxt[j];
            if (nxt[j] >= 0) prv[nxt[j]] = prv[j]; else tail = prv[j];
        };
        for (int32_t j : order) { append(j); ++valid; }
        for (uint64_t w = chunk_lo(c); w < chunk_lo(c + 1); ++w) {
            const int64_t idx = (int64_t)log.sym[w] - (int64_t)W;
            if (idx >= 0) {
                const int32_t j = (int32_t)((uint64_t)idx % W);
                if (lst[j] < 0) ++valid; else unlink(j);
                append(j);
                lst[j] = idx;
            }
            const int64_t imin = valid == W ? lst[head] : -1;
            const bool cand = idx >= 0 && valid == W && (uint64_t)(idx / W - imin / W) <= kMaxGroupDiff;
            key[w] = (uint32_t)(imin + 1) | (cand ? 0u : kNotCandidate);
        }
    });
    // Pass 3: the greedy choice (Def. 4.1) and the chosen words' backward scans.
    uint32_t k = 1;
    int64_t prev_max = -1, T = 0;
    auto retarget = [&] {
        const int64_t remaining = std::max<int64_t>(0, (int64_t)b.n_symbols - prev_max - 1);
        T = (int64_t)cdiv((uint64_t)remaining, M - k + 1);
    };
    retarget();
    std::vector<int64_t> snap_idx(W, -1), idx_of(W);
    std::vector<uint16_t> snap_state(W, 0);
    std::vector<uint8_t> seen(W);
    uint64_t floor = 0;   // first word after the previous chosen one
    auto imax_of = [&](uint64_t w) { return (int64_t)log.sym[w] - (int64_t)W; };
    auto imin_of = [&](uint64_t w) { return (int64_t)(key[w] & ~kNotCandidate) - 1; };
    auto is_cand = [&](uint64_t w) { return !(key[w] & kNotCandidate); };
    // First word in [lo, B) whose Imin exceeds v (Imin never falls), or B.
    auto first_imin_above = [&](uint64_t lo, int64_t v) {
        uint64_t l = lo, h = B;
        while (l < h) { const uint64_t m = l + (h - l) / 2; if (imin_of(m) > v) h = m; else l = m + 1; }
        return l;
    };
    // First word in [lo, B) whose Imax is at least v (Imax grows), or B.
    auto first_imax_from = [&](uint64_t lo, int64_t v) {
        uint64_t l = lo, h = B;
        while (l < h) { const uint64_t m = l + (h - l) / 2; if (imax_of(m) >= v) h = m; else l = m + 1; }
        return l;
    };
    auto choose = [&](uint64_t wb) {
        const int64_t imax = imax_of(wb);
        std::fill(seen.begin(), seen.end(), 0);
        const size_t base = b.sp_state.size();
        b.sp_state.resize(base + W);
        b.sp_gdiff.resize(base + W);
        uint32_t nseen = 0;
        for (uint64_t q = wb + 1; q > floor && nseen < W; --q) {
            const int64_t idx = imax_of(q - 1);
            if (idx < 0) continue;
            const uint32_t j = (uint32_t)((uint64_t)idx % W);
            if (seen[j]) continue;
            seen[j] = 1;
            ++nseen;
            idx_of[j] = idx;
            b.sp_state[base + j] = log.state[q - 1];
        }
        for (uint32_t j = 0; j < W; ++j) {
            if (!seen[j]) { idx_of[j] = snap_idx[j]; b.sp_state[base + j] = snap_state[j]; }
            snap_idx[j] = idx_of[j];
            snap_state[j] = b.sp_state[base + j];
        }
        const uint64_t anchor = (uint64_t)imax / W;
        for (uint32_t j = 0; j < W; ++j) b.sp_gdiff[base + j] = (uint16_t)(anchor - (uint64_t)idx_of[j] / W);
        b.sp_next.push_back(wb + 1);
        b.sp_anchor.push_back(anchor);
        floor = wb + 1;
        prev_max = imax;
        ++k;
        retarget();
    };
    while (k < M) {
        uint64_t lo = floor;
        while (lo < B && !is_cand(lo)) ++lo;
        if (lo >= B) break;
        const int64_t c = prev_max + T;
        // The window: candidates before the first one with t > 2T + t_s.
        uint64_t end = first_imin_above(lo, c + T + 1);
        while (end < B && !is_cand(end)) ++end;
        if (end == lo) { choose(lo); continue; }   // the first candidate already closes it
        bool have = false;
        uint64_t best = 0;
        int64_t best_h = 0;
        auto score = [&](uint64_t w) {
            const int64_t t = imax_of(w) - prev_max, ts = imax_of(w) - imin_of(w) + 1;
            const int64_t h = std::llabs(t - T) + std::llabs(t - ts - T);
            if (!have || h < best_h) { have = true; best = w; best_h = h; }
        };
        const uint64_t a_end = std::min(end, first_imax_from(lo, c));
        const uint64_t c_start = std::max(a_end, std::min(end, first_imin_above(lo, c + 1)));
        for (uint64_t w = a_end; w > lo; --w)
            if (is_cand(w - 1)) { score(w - 1); break; }    // the last falling candidate
        for (uint64_t w = a_end; w < c_start; ++w)
            if (is_cand(w)) score(w);                       // the level ones
        for (uint64_t w = c_start; w < end; ++w)
            if (is_cand(w)) { score(w); break; }            // the first rising one
        choose(best);
    }
}

// tidx: adaptive coding (symbol i with table tidx[i]), or NULL for the one table.
template <typename Sym>
void encode_stream(const Sym *sym, BlobData &b, uint32_t threads, const uint8_t *tidx = nullptr) {
    const uint32_t W = b.lanes, n = b.quant_bits, A = b.alphabet;
    std::vector<uint32_t> F((size_t)b.tables * (A + 1), 0);   // table t's cumulative counts at t (A + 1)
    for (uint32_t t = 0; t < b.tables; ++t)
        for (uint32_t s = 0; s < A; ++s) F[(size_t)t * (A + 1) + s + 1] = F[(size_t)t * (A + 1) + s] + b.freq[(size_t)t * A + s];
    SplitChooser chooser(b, threads);
    const bool want_splits = threads > 1;
    // The threaded writer keeps symbol indices and Imin + 1 in 31 bits.
    const uint32_t writers = want_splits && b.n_symbols < (1ull << 31) ? split_writer_threads(b.n_symbols) : 1u;
    EventLog log;
    if (writers > 1) {
        log.sym.reserve((size_t)(b.n_symbols / 2) + 16);
        log.state.reserve((size_t)(b.n_symbols / 2) + 16);
    }
    uint32_t x[64];
    for (uint32_t j = 0; j < W; ++j) x[j] = kLower;
    std::vector<uint16_t> &words = *b.words_buf;
    // Words per symbol are at most one (b >= n); reserve an estimate.
    words.reserve((size_t)(b.n_symbols / 2) + 16);
    const uint32_t shift = kLowerBits + kWordBits - n;   // threshold = ((L >> n) << b) * f
    uint32_t j = 0;
    for (uint64_t i = 0; i < b.n_symbols; ++i) {
        const uint32_t s = sym[i];
        const uint32_t t = tidx ? tidx[i] : 0u;
        const uint32_t fs = b.freq[(size_t)t * A + s];
        uint32_t xs = x[j];
        if ((uint64_t)xs >= ((uint64_t)fs << shift)) {
            // Emit the low word first, then shift (Eq. 3).
            words.push_back((uint16_t)(xs & 0xFFFFu));
            xs >>= kWordBits;
            if (writers > 1) {
                log.sym.push_back((uint32_t)i);
                log.state.push_back((uint16_t)xs);
            } else if (want_splits) {
                chooser.event(words.size() - 1, (int64_t)i - (int64_t)W, xs);
            }
        }
        x[j] = ((xs / fs) << n) + F[(size_t)t * (A + 1) + s] + (xs % fs);     // Eq. 1
        if (++j == W) j = 0;
    }
    if (writers > 1) choose_splits_parallel(b, log, threads, writers);
    else if (want_splits) chooser.finish();
    b.final_states.assign(x, x + W);
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }
recoil_status fail(recoil_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

bool pack_sections(BlobData &b) {
    b.table_bits.clear();
    b.meta_bits.clear();
    b.x_series_bit = 0;
    b.block_bit.clear();
    {
        // One series per table, back to back in one bit stream.
        BitSink s(b.table_bits);
        for (uint32_t t = 0; t < b.tables; ++t) {
            const uint64_t base = (uint64_t)t * b.alphabet;
            if (!put_series(s, b.alphabet, 5, false, [&](uint64_t k) { return (int64_t)b.freq[base + k]; }))
                return false;
        }
        s.flush();
    }
    if (b.partitioned()) {
        // Per sub-sequence: its first word, then its W final states (u32 each).
        const uint32_t W = b.lanes;
        b.meta_bits.reserve(b.part_start.size() * 4 * (1 + W));
        for (size_t q = 0; q < b.part_start.size(); ++q) {
            if (b.part_start[q] >= (1ull << 32)) return false;
            put_u(b.meta_bits, b.part_start[q], 4);
            for (uint32_t j = 0; j < W; ++j) put_u(b.meta_bits, b.part_final[q * W + j], 4);
        }
        return true;
    }
    const uint32_t M = b.splits();
    if (M == 1) return true;
    const uint64_t W = b.lanes;
    const uint64_t Eb = cdiv(b.n_words(), M);
    const uint64_t Eg = cdiv(b.groups(), M);
    BitSink s(b.meta_bits);
    if (!put_series(s, M - 1, 5, true, [&](uint64_t k) {
            return (int64_t)b.sp_next[k] - (int64_t)((k + 1) * Eb);
        }))
        return false;
    b.x_series_bit = s.bit_pos();
    if (!put_series(s, M - 1, 5, true, [&](uint64_t k) {
            return (int64_t)(b.sp_anchor[k] + 1) - (int64_t)((k + 1) * Eg);   // 1-based group ids
        }))
        return false;
    b.block_bit.assign(M - 1, 0);
    for (uint64_t k = 0; k + 1 < M; ++k) {
        b.block_bit[k] = s.bit_pos();
        for (uint64_t j = 0; j < W; ++j) s.put(b.sp_state[k * W + j], 16);
        if (!put_series(s, W, 4, false, [&](uint64_t j) { return (int64_t)b.sp_gdiff[k * W + j]; }))
            return false;
    }
    s.flush();
    return true;
}

recoil_status quantize(const uint64_t *counts, uint32_t A, uint32_t n, uint32_t *f_out) {
    if (!counts || !f_out || A == 0 || n < 1 || n > 16) return fail(RECOIL_ERR_INVALID_ARG, "quantize: bad arguments");
    const uint64_t total = 1ull << n;
    uint64_t N = 0, present = 0;
    for (uint32_t s = 0; s < A; ++s) { N += counts[s]; present += counts[s] != 0; }
    if (present == 0 || present > total) return fail(RECOIL_ERR_INFEASIBLE, "quantize: no symbol or more symbols than 2^n slots");
    std::vector<uint64_t> f(A, 0), rem(A, 0);
    uint64_t sum = 0;
    for (uint32_t s = 0; s < A; ++s) {
        if (!counts[s]) continue;
        unsigned __int128 scaled = (unsigned __int128)counts[s] * total;
        f[s] = (uint64_t)(scaled / N);
        rem[s] = (uint64_t)(scaled % N);
        if (!f[s]) f[s] = 1;
        sum += f[s];
    }
    if (sum < total) {
        std::vector<uint32_t> order;
        for (uint32_t s = 0; s < A; ++s) if (counts[s]) order.push_back(s);
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return rem[a] > rem[c]; });
        for (uint64_t k = 0; sum < total; ++k) { f[order[k]]++; ++sum; }
    }
    if (sum > total) {
        // Max-heap on (f, -s): largest f first, smaller symbol on ties.
        auto cmp = [&](uint32_t a, uint32_t c) { return f[a] != f[c] ? f[a] < f[c] : a > c; };
        std::priority_queue<uint32_t, std::vector<uint32_t>, decltype(cmp)> heap(cmp);
        for (uint32_t s = 0; s < A; ++s) if (f[s] > 1) heap.push(s);
        while (sum > total) {
            uint32_t s = heap.top();
            heap.pop();
            f[s]--;
            --sum;
            if (f[s] > 1) heap.push(s);
        }
    }
    for (uint32_t s = 0; s < A; ++s) f_out[s] = (uint32_t)f[s];
    return RECOIL_OK;
}

// Parameters, symbol check and table (given or quantised from the counts) of a new blob.
recoil_status prepare_blob(const void *symbols, uint64_t N, const recoil_config *cfg, const uint32_t *freq,
                           std::shared_ptr<BlobData> &out) {
    const uint32_t W = cfg->lanes, n = cfg->quant_bits, sb = cfg->symbol_bytes, A = cfg->alphabet;
    if (W < 1 || W > 64 || n < 1 || n > 16 || (sb != 1 && sb != 2) || A < 1 || A > (sb == 1 ? 256u : 65536u))
        return fail(RECOIL_ERR_INVALID_ARG, "encode: configuration out of range");
    auto b = std::make_shared<BlobData>();
    b->lanes = W; b->quant_bits = n; b->symbol_bytes = sb; b->alphabet = A; b->n_symbols = N;
    b->freq.assign(A, 0);
    std::vector<uint64_t> counts(A, 0);
    if (sb == 1) {
        const uint8_t *s = (const uint8_t *)symbols;
        for (uint64_t i = 0; i < N; ++i) { if (s[i] >= A) return fail(RECOIL_ERR_INVALID_ARG, "encode: symbol outside the alphabet"); counts[s[i]]++; }
    } else {
        const uint16_t *s = (const uint16_t *)symbols;
        for (uint64_t i = 0; i < N; ++i) { if (s[i] >= A) return fail(RECOIL_ERR_INVALID_ARG, "encode: symbol outside the alphabet"); counts[s[i]]++; }
    }
    if (freq) {
        uint64_t tot = 0;
        for (uint32_t s = 0; s < A; ++s) { b->freq[s] = freq[s]; tot += freq[s]; }
        if (tot != (1ull << n)) return fail(RECOIL_ERR_INVALID_ARG, "encode: freq does not sum to 2^n");
    } else if (N > 0) {
        recoil_status st = quantize(counts.data(), A, n, b->freq.data());
        if (st) return st;
    } else {
        b->freq[0] = 1u << n;
    }
    for (uint32_t s = 0; s < A; ++s)
        if (counts[s] && !b->freq[s]) return fail(RECOIL_ERR_INFEASIBLE, "encode: a present symbol has zero frequency");
    out = std::move(b);
    return RECOIL_OK;
}

recoil_status encode(const void *symbols, uint64_t N, const recoil_config *cfg, const uint32_t *freq,
                     uint32_t threads, recoil_blob **out) {
    if (!out) return fail(RECOIL_ERR_INVALID_ARG, "encode: out is NULL");
    *out = nullptr;
    if (!cfg || (N > 0 && !symbols) || threads < 1) return fail(RECOIL_ERR_INVALID_ARG, "encode: bad arguments");
    std::shared_ptr<BlobData> b;
    recoil_status st = prepare_blob(symbols, N, cfg, freq, b);
    if (st) return st;
    if (b->symbol_bytes == 1) encode_stream((const uint8_t *)symbols, *b, threads);
    else encode_stream((const uint16_t *)symbols, *b, threads);
    if (!pack_sections(*b)) return fail(RECOIL_ERR_INFEASIBLE, "encode: metadata does not fit its series");
    auto *h = new (std::nothrow) recoil_blob();
    if (!h) return fail(RECOIL_ERR_INVALID_ARG, "encode: out of memory");
    h->data = std::move(b);
    *out = h;
    return RECOIL_OK;
}

recoil_status encode_adaptive(const void *symbols, uint64_t N, const recoil_config *cfg, const uint32_t *freqs,
                              uint32_t tables, const uint8_t *tidx, uint32_t threads, recoil_blob **out) {
    if (!out) return fail(RECOIL_ERR_INVALID_ARG, "encode_adaptive: out is NULL");
    *out = nullptr;
    if (!cfg || (N > 0 && (!symbols || !tidx)) || !freqs || threads < 1 || tables < 1 || tables > 256)
        return fail(RECOIL_ERR_INVALID_ARG, "encode_adaptive: bad arguments");
    const uint32_t W = cfg->lanes, n = cfg->quant_bits, sb = cfg->symbol_bytes, A = cfg->alphabet;
    if (W < 1 || W > 64 || n < 1 || n > 16 || (sb != 1 && sb != 2) || A < 1 || A > (sb == 1 ? 256u : 65536u))
        return fail(RECOIL_ERR_INVALID_ARG, "encode_adaptive: configuration out of range");
    auto b = std::make_shared<BlobData>();
    b->lanes = W; b->quant_bits = n; b->symbol_bytes = sb; b->alphabet = A; b->n_symbols = N;
    b->adaptive = true;
    b->tables = tables;
    b->freq.assign(freqs, freqs + (size_t)tables * A);
    for (uint32_t t = 0; t < tables; ++t) {
        uint64_t tot = 0;
        for (uint32_t s = 0; s < A; ++s) tot += b->freq[(size_t)t * A + s];
        if (tot != (1ull << n)) return fail(RECOIL_ERR_INVALID_ARG, "encode_adaptive: a table does not sum to 2^n");
    }
    for (uint64_t i = 0; i < N; ++i) {
        const uint32_t s = sb == 1 ? ((const uint8_t *)symbols)[i] : ((const uint16_t *)symbols)[i];
        if (s >= A || tidx[i] >= tables) return fail(RECOIL_ERR_INVALID_ARG, "encode_adaptive: symbol or table index out of range");
        if (!b->freq[(size_t)tidx[i] * A + s]) return fail(RECOIL_ERR_INFEASIBLE, "encode_adaptive: symbol has zero frequency in its table");
    }
    if (sb == 1) encode_stream((const uint8_t *)symbols, *b, threads, tidx);
    else encode_stream((const uint16_t *)symbols, *b, threads, tidx);
    if (!pack_sections(*b)) return fail(RECOIL_ERR_INFEASIBLE, "encode_adaptive: metadata does not fit its series");
    auto *h = new (std::nothrow) recoil_blob();
    if (!h) return fail(RECOIL_ERR_INVALID_ARG, "encode_adaptive: out of memory");
    h->data = std::move(b);
    *out = h;
    return RECOIL_OK;
}

namespace {

// One sub-sequence of the conventional baseline: W interleaved coders from state L
// over symbols [lo, hi) (whole groups from lo, so lane = (i - lo) mod W = i mod W).
template <typename Sym>
void encode_part(const Sym *sym, uint64_t lo, uint64_t hi, const std::vector<uint32_t> &F, BlobData &b) {
    const uint32_t W = b.lanes, n = b.quant_bits;
    const uint32_t shift = kLowerBits + kWordBits - n;
    std::vector<uint16_t> &words = *b.words_buf;
    uint32_t x[64];
    for (uint32_t j = 0; j < W; ++j) x[j] = kLower;
    uint32_t j = 0;
    for (uint64_t i = lo; i < hi; ++i) {
        const uint32_t s = sym[i], fs = b.freq[s];
        uint32_t xs = x[j];
        if ((uint64_t)xs >= ((uint64_t)fs << shift)) {
            words.push_back((uint16_t)(xs & 0xFFFFu));
            xs >>= kWordBits;
        }
        x[j] = ((xs / fs) << n) + F[s] + (xs % fs);
        if (++j == W) j = 0;
    }
    b.part_final.insert(b.part_final.end(), x, x + W);
}

}  // namespace

recoil_status encode_partitioned(const void *symbols, uint64_t N, const recoil_config *cfg, const uint32_t *freq,
                                 uint32_t partitions, recoil_blob **out) {
    if (!out) return fail(RECOIL_ERR_INVALID_ARG, "encode_partitioned: out is NULL");
    *out = nullptr;
    if (!cfg || (N > 0 && !symbols) || partitions < 1)
        return fail(RECOIL_ERR_INVALID_ARG, "encode_partitioned: bad arguments");
    std::shared_ptr<BlobData> b;
    recoil_status st = prepare_blob(symbols, N, cfg, freq, b);
    if (st) return st;
    const uint64_t W = b->lanes;
    const uint64_t S = std::max<uint64_t>(1, cdiv(std::max<uint64_t>(cdiv(N, partitions), 1), W)) * W;
    const uint64_t P = std::max<uint64_t>(1, cdiv(N, S));
    if (S >= (1ull << 32) || P >= (1ull << 32)) return fail(RECOIL_ERR_UNSUPPORTED, "encode_partitioned: too large");
    std::vector<uint32_t> F(b->alphabet + 1, 0);
    for (uint32_t s = 0; s < b->alphabet; ++s) F[s + 1] = F[s] + b->freq[s];
    b->part_size = S;
    b->words_buf->reserve((size_t)(N / 2) + 16);
    for (uint64_t q = 0; q < P; ++q) {
        const uint64_t lo = q * S, hi = std::min<uint64_t>(N, lo + S);
        b->part_start.push_back(b->n_words());
        if (b->symbol_bytes == 1) encode_part((const uint8_t *)symbols, lo, hi, F, *b);
        else encode_part((const uint16_t *)symbols, lo, hi, F, *b);
    }
    if (b->n_words() >= (1ull << 32) || !pack_sections(*b))
        return fail(RECOIL_ERR_UNSUPPORTED, "encode_partitioned: bitstream too long for the offset table");
    auto *h = new (std::nothrow) recoil_blob();
    if (!h) return fail(RECOIL_ERR_INVALID_ARG, "encode_partitioned: out of memory");
    h->data = std::move(b);
    *out = h;
    return RECOIL_OK;
}

std::shared_ptr<BlobData> combine_data(const BlobData &a, uint32_t target) {
    const uint32_t M = a.splits();
    const uint32_t step = (uint32_t)cdiv(M, std::min(std::max(target, 1u), M));
    auto b = std::make_shared<BlobData>();
    b->lanes = a.lanes; b->quant_bits = a.quant_bits; b->symbol_bytes = a.symbol_bytes;
    b->alphabet = a.alphabet; b->n_symbols = a.n_symbols;
    b->freq = a.freq; b->final_states = a.final_states; b->words_buf = a.words_buf;
    b->adaptive = a.adaptive; b->tables = a.tables;
    const uint64_t W = a.lanes;
    const size_t kept = M / step;
    b->sp_next.reserve(kept); b->sp_anchor.reserve(kept);
    b->sp_state.reserve(kept * W); b->sp_gdiff.reserve(kept * W);
    for (uint64_t k = step; k < M; k += step) {
        b->sp_next.push_back(a.sp_next[k - 1]);
        b->sp_anchor.push_back(a.sp_anchor[k - 1]);
        b->sp_state.insert(b->sp_state.end(), a.sp_state.begin() + (k - 1) * W, a.sp_state.begin() + k * W);
        b->sp_gdiff.insert(b->sp_gdiff.end(), a.sp_gdiff.begin() + (k - 1) * W, a.sp_gdiff.begin() + k * W);
    }
    if (!pack_sections(*b)) return nullptr;
    return b;
}

recoil_status combine(const recoil_blob *in, uint32_t target, recoil_blob **out) {
    if (!in || !out || target < 1) return fail(RECOIL_ERR_INVALID_ARG, "combine: bad arguments");
    *out = nullptr;
    if (in->data->partitioned())
        return fail(RECOIL_ERR_UNSUPPORTED, "combine: sub-sequences of a partitioned stream cannot be merged");
    std::shared_ptr<BlobData> b = combine_data(*in->data, target);
    if (!b) return fail(RECOIL_ERR_INFEASIBLE, "combine: metadata does not fit its series");
    auto *h = new (std::nothrow) recoil_blob();
    if (!h) return fail(RECOIL_ERR_INVALID_ARG, "combine: out of memory");
    h->data = std::move(b);
    *out = h;
    return RECOIL_OK;
}

recoil_status serialize(const recoil_blob *blob, void *dst, size_t cap, size_t *written) {
    if (!blob || !written) return fail(RECOIL_ERR_INVALID_ARG, "serialize: bad arguments");
    const BlobData &b = *blob->data;
    const uint64_t total = b.total_bytes();
    *written = (size_t)total;
    if (!dst) return RECOIL_OK;
    if (cap < total) return fail(RECOIL_ERR_BUFFER_TOO_SMALL, "serialize: destination too small");
    std::vector<uint8_t> h;
    h.reserve(48);
    h.push_back('R'); h.push_back('C'); h.push_back(b.partitioned() ? 'P' : b.adaptive ? 'A' : 'L'); h.push_back('1');
    put_u(h, 1, 2);
    h.push_back((uint8_t)b.lanes); h.push_back((uint8_t)b.quant_bits); h.push_back((uint8_t)b.symbol_bytes);
    h.push_back((uint8_t)kLowerBits); h.push_back((uint8_t)kWordBits); h.push_back(0);
    put_u(h, b.alphabet, 4);
    put_u(h, b.n_symbols, 8);
    put_u(h, b.n_words(), 8);
    put_u(h, b.splits(), 4);
    put_u(h, b.table_bits.size(), 4);
    put_u(h, b.meta_bits.size(), 4);
    put_u(h, b.partitioned() ? b.part_size : b.adaptive ? b.tables : 0, 4);
    uint8_t *p = (uint8_t *)dst;
    std::memcpy(p, h.data(), 48);
    p += 48;
    std::memcpy(p, b.table_bits.data(), b.table_bits.size());
    p += b.table_bits.size();
    if (!b.partitioned())
        for (uint32_t x : b.final_states) { for (int k = 0; k < 4; ++k) *p++ = (uint8_t)(x >> (8 * k)); }
    if (!b.meta_bits.empty()) std::memcpy(p, b.meta_bits.data(), b.meta_bits.size());
    p += b.meta_bits.size();
    for (uint16_t w : *b.words_buf) { *p++ = (uint8_t)w; *p++ = (uint8_t)(w >> 8); }
    return RECOIL_OK;
}

namespace {

// The table section: f[s] as a bit series summing to 2^n (Sec. 4.4).
recoil_status parse_table(const uint8_t *q, uint64_t tbytes, BlobData &b) {
    BitSource s(q, tbytes);
    std::vector<int64_t> fv;
    if (!get_series(s, b.alphabet, 5, false, fv) || cdiv(s.pos(), 8) != tbytes)
        return fail(RECOIL_ERR_CORRUPT, "container: bad table");
    uint64_t tot = 0;
    b.freq.resize(b.alphabet);
    for (uint32_t k = 0; k < b.alphabet; ++k) {
        if (fv[k] > (int64_t)(1u << b.quant_bits)) return fail(RECOIL_ERR_CORRUPT, "container: bad table");
        b.freq[k] = (uint32_t)fv[k];
        tot += (uint64_t)fv[k];
    }
    if (tot != (1ull << b.quant_bits)) return fail(RECOIL_ERR_CORRUPT, "container: table does not sum to 2^n");
    return RECOIL_OK;
}

// Conventional container ("RCP1"): the header's thread field counts sub-sequences,
// its last word is the sub-sequence length S; per sub-sequence its first word and
// W final states follow the table; then the words.
recoil_status deserialize_partitioned(const uint8_t *c, size_t len, recoil_blob **out) {
    auto b = std::make_shared<BlobData>();
    b->lanes = c[6]; b->quant_bits = c[7]; b->symbol_bytes = c[8];
    const uint32_t lbits = c[9], wbits = c[10];
    b->alphabet = (uint32_t)get_u(c + 12, 4);
    b->n_symbols = get_u(c + 16, 8);
    const uint64_t B = get_u(c + 24, 8), P = get_u(c + 32, 4);
    const uint64_t tbytes = get_u(c + 36, 4), mbytes = get_u(c + 40, 4), S = get_u(c + 44, 4);
    const uint32_t W = b->lanes, n = b->quant_bits, sb = b->symbol_bytes, A = b->alphabet;
    if (c[11] != 0) return fail(RECOIL_ERR_CORRUPT, "container: reserved byte set");
    if (W < 1 || W > 64 || n < 1 || n > 16 || (sb != 1 && sb != 2) || A < 1 || A > (sb == 1 ? 256u : 65536u))
        return fail(RECOIL_ERR_CORRUPT, "container: parameters out of range");
    if (lbits != kLowerBits || wbits != kWordBits) return fail(RECOIL_ERR_UNSUPPORTED, "container: only L = 2^16, b = 16 supported");
    if (S == 0 || S % W || P != std::max<uint64_t>(1, cdiv(b->n_symbols, S)))
        return fail(RECOIL_ERR_CORRUPT, "container: sub-sequence length and count disagree");
    if (B > len / 2 || tbytes > len || mbytes != P * 4 * (1 + (uint64_t)W) || 48 + tbytes + mbytes + 2 * B != len)
        return fail(RECOIL_ERR_CORRUPT, "container: length mismatch");
    const uint8_t *q = c + 48;
    recoil_status st = parse_table(q, tbytes, *b);
    if (st) return st;
    q += tbytes;
    b->part_size = S;
    b->part_start.resize(P);
    b->part_final.resize(P * W);
    for (uint64_t k = 0; k < P; ++k) {
        b->part_start[k] = get_u(q, 4);
        q += 4;
        if ((k == 0 && b->part_start[0] != 0) || b->part_start[k] > B || (k && b->part_start[k] < b->part_start[k - 1]))
            return fail(RECOIL_ERR_CORRUPT, "container: sub-bitstream offsets not increasing inside the bitstream");
        for (uint32_t j = 0; j < W; ++j, q += 4) {
            b->part_final[k * W + j] = (uint32_t)get_u(q, 4);
            if (b->part_final[k * W + j] < kLower) return fail(RECOIL_ERR_CORRUPT, "container: final state below L");
        }
    }
    std::vector<uint16_t> &words = *b->words_buf;
    words.resize(B);
    for (uint64_t k = 0; k < B; ++k) words[k] = (uint16_t)(q[2 * k] | (q[2 * k + 1] << 8));
    if (!pack_sections(*b) || b->table_bits.size() != tbytes || b->meta_bits.size() != mbytes)
        return fail(RECOIL_ERR_CORRUPT, "container: non-canonical table series");
    auto *h = new (std::nothrow) recoil_blob();
    if (!h) return fail(RECOIL_ERR_INVALID_ARG, "deserialize: out of memory");
    h->data = std::move(b);
    *out = h;
    return RECOIL_OK;
}

}  // namespace

recoil_status deserialize(const void *src, size_t len, recoil_blob **out) {
    if (!src || !out) return fail(RECOIL_ERR_INVALID_ARG, "deserialize: bad arguments");
    *out = nullptr;
    const uint8_t *c = (const uint8_t *)src;
    if (len >= 48 && std::memcmp(c, "RCP1", 4) == 0) {
        if (get_u(c + 4, 2) != 1) return fail(RECOIL_ERR_CORRUPT, "container: unknown version");
        return deserialize_partitioned(c, len, out);
    }
    const bool adaptive = len >= 48 && std::memcmp(c, "RCA1", 4) == 0;
    if (len < 48 || (!adaptive && std::memcmp(c, "RCL1", 4) != 0)) return fail(RECOIL_ERR_CORRUPT, "container: bad magic");
    if (get_u(c + 4, 2) != 1) return fail(RECOIL_ERR_CORRUPT, "container: unknown version");
    auto b = std::make_shared<BlobData>();
    b->adaptive = adaptive;
    b->tables = adaptive ? (uint32_t)get_u(c + 44, 4) : 1u;
    if (b->tables < 1 || b->tables > 256) return fail(RECOIL_ERR_CORRUPT, "container: table count out of range");
    b->lanes = c[6]; b->quant_bits = c[7]; b->symbol_bytes = c[8];
    const uint32_t lbits = c[9], wbits = c[10];
    b->alphabet = (uint32_t)get_u(c + 12, 4);
    b->n_symbols = get_u(c + 16, 8);
    const uint64_t B = get_u(c + 24, 8);
    const uint64_t M = get_u(c + 32, 4);
    const uint64_t tbytes = get_u(c + 36, 4), mbytes = get_u(c + 40, 4);
    const uint32_t W = b->lanes, n = b->quant_bits, sb = b->symbol_bytes, A = b->alphabet;
    if (c[11] != 0 || (!adaptive && get_u(c + 44, 4) != 0)) return fail(RECOIL_ERR_CORRUPT, "container: reserved bytes set");
    if (W < 1 || W > 64 || n < 1 || n > 16 || (sb != 1 && sb != 2) || A < 1 || A > (sb == 1 ? 256u : 65536u))
        return fail(RECOIL_ERR_CORRUPT, "container: parameters out of range");
    if (lbits != kLowerBits || wbits != kWordBits) return fail(RECOIL_ERR_UNSUPPORTED, "container: only L = 2^16, b = 16 supported");
    if (M < 1) return fail(RECOIL_ERR_CORRUPT, "container: zero splits");
    if (B > len / 2 || tbytes > len || mbytes > len) return fail(RECOIL_ERR_CORRUPT, "container: section sizes exceed length");
    if (48 + tbytes + 4ull * W + mbytes + 2 * B != len) return fail(RECOIL_ERR_CORRUPT, "container: length mismatch");
    // Every split point carries W 16-bit states, so the metadata size bounds M (and
    // what is allocated below). Split points may share a symbol group: a stream
    // cut finer than its groups has more units than groups, some of them empty.
    if ((M - 1) * 2ull * W > mbytes) return fail(RECOIL_ERR_CORRUPT, "container: more splits than the metadata holds");
    const uint8_t *q = c + 48;
    {
        BitSource s(q, tbytes);
        b->freq.resize((size_t)b->tables * A);
        for (uint32_t t = 0; t < b->tables; ++t) {
            std::vector<int64_t> fv;
            if (!get_series(s, A, 5, false, fv)) return fail(RECOIL_ERR_CORRUPT, "container: bad table");
            uint64_t tot = 0;
            for (uint32_t k = 0; k < A; ++k) {
                if (fv[k] > (int64_t)(1u << n)) return fail(RECOIL_ERR_CORRUPT, "container: bad table");
                b->freq[(size_t)t * A + k] = (uint32_t)fv[k];
                tot += (uint64_t)fv[k];
            }
            if (tot != (1ull << n)) return fail(RECOIL_ERR_CORRUPT, "container: table does not sum to 2^n");
        }
        if (cdiv(s.pos(), 8) != tbytes) return fail(RECOIL_ERR_CORRUPT, "container: bad table");
    }
    q += tbytes;
    b->final_states.resize(W);
    for (uint32_t j = 0; j < W; ++j) {
        b->final_states[j] = (uint32_t)get_u(q + 4 * j, 4);
        if (b->final_states[j] < kLower) return fail(RECOIL_ERR_CORRUPT, "container: final state below L");
    }
    q += 4ull * W;
    if (M > 1) {
        const uint64_t G = b->groups();
        const uint64_t Eb = cdiv(B, M), Eg = cdiv(G, M);
        BitSource s(q, mbytes);
        std::vector<int64_t> O, X;
        if (!get_series(s, M - 1, 5, true, O) || !get_series(s, M - 1, 5, true, X))
            return fail(RECOIL_ERR_CORRUPT, "container: bad split series");
        b->sp_next.resize(M - 1);
        b->sp_anchor.resize(M - 1);
        b->sp_state.resize((M - 1) * W);
        b->sp_gdiff.resize((M - 1) * W);
        std::vector<int64_t> d;
        uint64_t prev_next = 0, prev_min = 0;
        for (uint64_t k = 1; k < M; ++k) {
            const int64_t next = O[k - 1] + (int64_t)(k * Eb);
            const int64_t anchor = X[k - 1] + (int64_t)(k * Eg) - 1;
            if (next < 1 || (uint64_t)next > B || next <= (int64_t)prev_next)
                return fail(RECOIL_ERR_CORRUPT, "container: split offsets not increasing inside the bitstream");
            if (anchor < 0 || (uint64_t)anchor >= G) return fail(RECOIL_ERR_CORRUPT, "container: anchor group out of range");
            b->sp_next[k - 1] = (uint64_t)next;
            b->sp_anchor[k - 1] = (uint64_t)anchor;
            for (uint32_t j = 0; j < W; ++j) {
                uint64_t v;
                if (!s.get(16, v)) return fail(RECOIL_ERR_CORRUPT, "container: truncated split states");
                if (v == 0) return fail(RECOIL_ERR_CORRUPT, "container: zero split state");
                b->sp_state[(k - 1) * W + j] = (uint16_t)v;
            }
            if (!get_series(s, W, 4, false, d)) return fail(RECOIL_ERR_CORRUPT, "container: bad group series");
            int64_t mind = INT64_MAX;
            uint64_t imin = UINT64_MAX, imax = 0;
            for (uint32_t j = 0; j < W; ++j) {
                if (d[j] > anchor) return fail(RECOIL_ERR_CORRUPT, "container: group difference beyond anchor");
                mind = std::min(mind, d[j]);
                b->sp_gdiff[(k - 1) * W + j] = (uint16_t)d[j];
                uint64_t idx = (uint64_t)(anchor - d[j]) * W + j;
                imin = std::min(imin, idx);
                imax = std::max(imax, idx);
            }
            if (mind != 0) return fail(RECOIL_ERR_CORRUPT, "container: anchor is not the largest group");
            if (imax >= b->n_symbols) return fail(RECOIL_ERR_CORRUPT, "container: split index beyond N");
            if (imin < prev_min) return fail(RECOIL_ERR_CORRUPT, "container: split synchronisation points not monotone");
            prev_next = (uint64_t)next;
            prev_min = imin;
        }
        if (cdiv(s.pos(), 8) != mbytes) return fail(RECOIL_ERR_CORRUPT, "container: metadata length mismatch");
    } else if (mbytes != 0) {
        return fail(RECOIL_ERR_CORRUPT, "container: metadata present with one split");
    }
    q += mbytes;
    std::vector<uint16_t> &words = *b->words_buf;
    words.resize(B);
    for (uint64_t k = 0; k < B; ++k) words[k] = (uint16_t)(q[2 * k] | (q[2 * k + 1] << 8));
    if (!pack_sections(*b)) return fail(RECOIL_ERR_CORRUPT, "container: does not re-pack");
    if (b->table_bits.size() != tbytes || b->meta_bits.size() != mbytes)
        return fail(RECOIL_ERR_CORRUPT, "container: non-canonical series widths");
    auto *h = new (std::nothrow) recoil_blob();
    if (!h) return fail(RECOIL_ERR_INVALID_ARG, "deserialize: out of memory");
    h->data = std::move(b);
    *out = h;
    return RECOIL_OK;
}

}  // namespace recoil

extern "C" {

const char *recoil_status_string(recoil_status s) {
    switch (s) {
    case RECOIL_OK: return "ok";
    case RECOIL_ERR_INVALID_ARG: return "invalid argument";
    case RECOIL_ERR_INFEASIBLE: return "infeasible";
    case RECOIL_ERR_CORRUPT: return "corrupt container";
    case RECOIL_ERR_UNSUPPORTED: return "unsupported";
    case RECOIL_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case RECOIL_ERR_HIP: return "HIP error";
    case RECOIL_ERR_ALIGNMENT: return "misaligned pointer";
    case RECOIL_ERR_BUSY: return "busy";
    case RECOIL_ERR_NOT_FOUND: return "not found";
    case RECOIL_ERR_OUT_OF_MEMORY: return "out of host memory";
    default: return "unknown status";
    }
}

const char *recoil_last_error(void) { return recoil::g_last_error.c_str(); }
const char *recoil_version(void) { return "librecoil 0.1 (gfx950)"; }

recoil_status recoil_quantize(const uint64_t *counts, uint32_t alphabet, uint32_t quant_bits, uint32_t *f_out) {
    return recoil::guarded("quantize", [&]() -> recoil_status {
    return recoil::quantize(counts, alphabet, quant_bits, f_out);
    });
}

recoil_status recoil_encode(const void *symbols, uint64_t n_symbols, const recoil_config *cfg,
                            const uint32_t *freq, uint32_t n_splits, recoil_blob **out) {
    return recoil::guarded("encode", [&]() -> recoil_status {
    return recoil::encode(symbols, n_symbols, cfg, freq, n_splits, out);
    });
}

recoil_status recoil_encode_adaptive(const void *symbols, uint64_t n_symbols, const recoil_config *cfg,
                                     const uint32_t *freqs, uint32_t tables, const uint8_t *table_index,
                                     uint32_t n_splits, recoil_blob **out) {
    return recoil::guarded("encode_adaptive", [&]() -> recoil_status {
    return recoil::encode_adaptive(symbols, n_symbols, cfg, freqs, tables, table_index, n_splits, out);
    });
}

recoil_status recoil_encode_partitioned(const void *symbols, uint64_t n_symbols, const recoil_config *cfg,
                                        const uint32_t *freq, uint32_t partitions, recoil_blob **out) {
    return recoil::guarded("encode_partitioned", [&]() -> recoil_status {
    return recoil::encode_partitioned(symbols, n_symbols, cfg, freq, partitions, out);
    });
}

void recoil_set_split_writer_threads(uint32_t threads) {
    recoil::g_split_threads.store(threads, std::memory_order_relaxed);
}

recoil_status recoil_combine_splits(const recoil_blob *in, uint32_t target_splits, recoil_blob **out) {
    return recoil::guarded("combine_splits", [&]() -> recoil_status {
    return recoil::combine(in, target_splits, out);
    });
}

recoil_status recoil_blob_serialize(const recoil_blob *blob, void *dst, size_t cap, size_t *written) {
    return recoil::guarded("blob_serialize", [&]() -> recoil_status {
    return recoil::serialize(blob, dst, cap, written);
    });
}

recoil_status recoil_blob_deserialize(const void *src, size_t len, recoil_blob **out) {
    return recoil::guarded("blob_deserialize", [&]() -> recoil_status {
    return recoil::deserialize(src, len, out);
    });
}

recoil_status recoil_blob_info(const recoil_blob *blob, recoil_blob_info_t *out) {
    if (!blob || !out) return recoil::fail(RECOIL_ERR_INVALID_ARG, "blob_info: bad arguments");
    const recoil::BlobData &b = *blob->data;
    out->n_symbols = b.n_symbols;
    out->n_words = b.n_words();
    out->splits = b.splits();
    out->lanes = b.lanes;
    out->quant_bits = b.quant_bits;
    out->symbol_bytes = b.symbol_bytes;
    out->alphabet = b.alphabet;
    out->table_bytes = b.table_bits.size();
    out->metadata_bytes = b.meta_bits.size();
    out->total_bytes = b.total_bytes();
    return RECOIL_OK;
}

void recoil_blob_free(recoil_blob *blob) { delete blob; }

}  // extern "C"
