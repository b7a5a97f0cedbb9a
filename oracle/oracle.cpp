/*
 * Recoil CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain serial C++17, written from the paper's definitions:
 *   Eq. 1 / Eq. 2   rANS encode / decode step                (Sec. 2.1, Def. 2.1)
 *   Eq. 3 / Eq. 4   encoder / decoder renormalisation         (Sec. 2.1, Def. 2.2)
 *   Sec. 2.2        interleaved rANS (word order across lanes)
 *   Sec. 4.1        backward scan, synchronisation / decoding / cross-boundary phases
 *   Def. 4.1        split-selection heuristic H(t, t_s)
 *   Sec. 3.3, 4.2   split combining (keep every ceil(M_in/M_out)-th split point)
 *   Sec. 4.3        metadata storage (differences from rounded-up averages,
 *                   anchors, bit-packed series with a width field)
 * No blocking, no SIMD, no lookup tables: each step is written the way the
 * paper states it, so that it can be checked against the text by eye.
 */
#include "oracle.h"

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

// --------------------------------------------------------------------------
// Bit-packed series (Sec. 4.3): a (width-1) field, then each value with that
// many bits, MSB first; signed series add one sign bit per value.
// --------------------------------------------------------------------------
struct BitWriter {
    std::vector<uint8_t> bytes;
    uint64_t nbits = 0;
    void put(uint64_t value, uint32_t width) {
        for (int k = (int)width - 1; k >= 0; --k) {
            uint32_t bit = (uint32_t)((value >> k) & 1u);
            if (nbits % 8 == 0) bytes.push_back(0);
            if (bit) bytes.back() |= (uint8_t)(0x80u >> (nbits % 8));
            ++nbits;
        }
    }
};

struct BitReader {
    const uint8_t *data;
    uint64_t nbytes;
    uint64_t pos = 0;
    bool overrun = false;
    uint64_t get(uint32_t width) {
        uint64_t v = 0;
        for (uint32_t k = 0; k < width; ++k) {
            if (pos >= nbytes * 8) { overrun = true; return 0; }
            uint32_t bit = (data[pos / 8] >> (7 - pos % 8)) & 1u;
            v = (v << 1) | bit;
            ++pos;
        }
        return v;
    }
};

uint32_t bit_length(uint64_t v) {
    uint32_t n = 0;
    while (v) { ++n; v >>= 1; }
    return n;
}

// Returns false when a value does not fit the width field.
bool put_series(BitWriter &w, const std::vector<int64_t> &values, uint32_t width_field,
                bool is_signed) {
    uint32_t width = 1;  // zero still takes one bit (footnote to Sec. 4.3)
    for (int64_t v : values) {
        uint64_t mag = v < 0 ? (uint64_t)(-v) : (uint64_t)v;
        if (!is_signed && v < 0) return false;
        width = std::max(width, bit_length(mag));
    }
    if (width - 1 >= (1u << width_field)) return false;
    w.put(width - 1, width_field);
    for (int64_t v : values) {
        uint64_t mag = v < 0 ? (uint64_t)(-v) : (uint64_t)v;
        if (is_signed) w.put(v < 0 ? 1 : 0, 1);
        w.put(mag, width);
    }
    return true;
}

bool get_series(BitReader &r, uint64_t count, uint32_t width_field, bool is_signed,
                std::vector<int64_t> &out) {
    uint32_t width = (uint32_t)r.get(width_field) + 1;
    out.assign(count, 0);
    for (uint64_t k = 0; k < count; ++k) {
        bool neg = is_signed ? r.get(1) != 0 : false;
        uint64_t mag = r.get(width);
        out[k] = neg ? -(int64_t)mag : (int64_t)mag;
    }
    return !r.overrun;
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return b == 0 ? 0 : (a + b - 1) / b; }

void put_le(std::vector<uint8_t> &v, uint64_t x, int bytes) {
    for (int k = 0; k < bytes; ++k) v.push_back((uint8_t)(x >> (8 * k)));
}
uint64_t get_le(const uint8_t *p, int bytes) {
    uint64_t x = 0;
    for (int k = 0; k < bytes; ++k) x |= (uint64_t)p[k] << (8 * k);
    return x;
}

bool params_ok(const orc_params &p) {
    if (p.lanes < 1 || p.lanes > 64) return false;
    if (p.symbol_bytes != 1 && p.symbol_bytes != 2) return false;
    if (p.alphabet < 1 || p.alphabet > (p.symbol_bytes == 1 ? 256u : 65536u)) return false;
    if (p.quant_bits < 1 || p.quant_bits > 16) return false;
    if (p.l_bits < p.quant_bits || p.l_bits > 16) return false;     // L = k * 2^n
    if (p.b_bits < p.quant_bits || p.b_bits > 16) return false;     // one-step renormalisation
    if (p.l_bits + p.b_bits > 32) return false;                     // states fit 32 bits
    return true;
}

uint32_t symbol_at(const void *s, uint32_t bytes, uint64_t i) {
    return bytes == 1 ? ((const uint8_t *)s)[i] : ((const uint16_t *)s)[i];
}
void store_symbol(void *s, uint32_t bytes, uint64_t i, uint32_t v) {
    if (bytes == 1) ((uint8_t *)s)[i] = (uint8_t)v;
    else ((uint16_t *)s)[i] = (uint16_t)v;
}

// One split point as the decoder sees it (0-based symbol indices).
struct Split {
    uint64_t pos = 0;                 // word position of the split (first word read)
    std::vector<uint32_t> state;      // per lane: recorded post-shift state
    std::vector<int64_t> index;       // per lane: symbol index of that state
    int64_t imax() const { return *std::max_element(index.begin(), index.end()); }
    int64_t imin() const { return *std::min_element(index.begin(), index.end()); }
};

struct Stream {
    orc_params p{};
    uint64_t N = 0;
    std::vector<uint32_t> f;          // quantised PDF f(s)
    std::vector<uint16_t> words;      // bitstream B, written forward
    std::vector<uint32_t> final_state;
    std::vector<Split> splits;        // M-1 split points, increasing position
    // Conventional partitioning (Sec. 2.3) instead of split points when part_size > 0:
    // sub-sequence q holds symbols [q S, min((q + 1) S, N)) (S = part_size, a multiple
    // of W), coded on its own; its words start at part_start[q] and its final states
    // are part_final[q W .. q W + W - 1].
    uint64_t part_size = 0;
    std::vector<uint64_t> part_start;
    std::vector<uint32_t> part_final;
    // Adaptive coding (Sec. 3.1, third advantage of storing symbol indices): `tables`
    // frequency tables (f holds tables x A entries) and symbol i coded with table
    // tidx[i]. The index array is side information both ends hold (as a hyperprior
    // would give it); it is not part of the container.
    bool adaptive = false;
    uint32_t tables = 1;
    std::vector<uint8_t> tidx;
    uint32_t threads() const { return part_size ? (uint32_t)part_start.size() : (uint32_t)splits.size() + 1; }
    uint64_t groups() const { return ceil_div(N, p.lanes); }
    uint32_t table_of(uint64_t i) const { return adaptive ? tidx[i] : 0u; }
};


// Cumulative F(s) = sum_{t < s} f(t) (Def. 2.1).
std::vector<uint64_t> cdf_of(const std::vector<uint32_t> &f) {
    std::vector<uint64_t> F(f.size() + 1, 0);
    for (size_t s = 0; s < f.size(); ++s) F[s + 1] = F[s] + f[s];
    return F;
}

// Per-table f and F of a stream (one table unless it is adaptive).
void tables_of(const Stream &st, std::vector<std::vector<uint32_t>> &fs, std::vector<std::vector<uint64_t>> &Fs) {
    const uint32_t A = st.p.alphabet;
    fs.assign(st.tables, {});
    Fs.assign(st.tables, {});
    for (uint32_t t = 0; t < st.tables; ++t) {
        fs[t].assign(st.f.begin() + (size_t)t * A, st.f.begin() + (size_t)(t + 1) * A);
        Fs[t] = cdf_of(fs[t]);
    }
}

// ---------------------------------------------------------------------------
// Container serialisation (layout documented in include/recoil.h)
// ---------------------------------------------------------------------------
bool write_metadata(const Stream &st, std::vector<uint8_t> &out) {
    out.clear();
    const uint32_t M = st.threads();
    if (M == 1) return true;
    const uint64_t W = st.p.lanes;
    const uint64_t B = st.words.size();
    const uint64_t G = st.groups();
    const uint64_t Eb = ceil_div(B, M);   // expected sub-bitstream length (Sec. 4.3)
    const uint64_t Eg = ceil_div(G, M);   // expected max symbol group id (rounded-up average)
    std::vector<int64_t> O, X;
    for (uint32_t k = 1; k < M; ++k) {
        const Split &sp = st.splits[k - 1];
        O.push_back((int64_t)(sp.pos + 1) - (int64_t)(k * Eb));
        // Symbol group ids are 1-based in the paper (group of 1-based index i is ceil(i/W)).
        X.push_back((int64_t)(sp.imax() / (int64_t)W) + 1 - (int64_t)(k * Eg));
    }
    BitWriter w;
    if (!put_series(w, O, 5, true)) return false;
    if (!put_series(w, X, 5, true)) return false;
    for (uint32_t k = 1; k < M; ++k) {
        const Split &sp = st.splits[k - 1];
        int64_t anchor = sp.imax() / (int64_t)W;
        for (uint64_t j = 0; j < W; ++j) w.put(sp.state[j], 16);
        std::vector<int64_t> d;
        for (uint64_t j = 0; j < W; ++j) d.push_back(anchor - sp.index[j] / (int64_t)W);
        if (!put_series(w, d, 4, false)) return false;
    }
    out = w.bytes;
    return true;
}

// Conventional container: the same 48-byte header with magic "RCP1", the number of
// sub-sequences in the thread field and the sub-sequence length S in the last
// header word; the table; then per sub-sequence its first word (u32) and W final
// states (u32 each); then the concatenated words.
bool write_partitioned(const Stream &st, std::vector<uint8_t> &out) {
    BitWriter table;
    std::vector<int64_t> fv(st.f.begin(), st.f.end());
    if (!put_series(table, fv, 5, false)) return false;
    const uint32_t P = st.threads(), W = st.p.lanes;
    out.clear();
    out.push_back('R'); out.push_back('C'); out.push_back('P'); out.push_back('1');
    put_le(out, 1, 2);
    out.push_back((uint8_t)W);
    out.push_back((uint8_t)st.p.quant_bits);
    out.push_back((uint8_t)st.p.symbol_bytes);
    out.push_back((uint8_t)st.p.l_bits);
    out.push_back((uint8_t)st.p.b_bits);
    out.push_back(0);
    put_le(out, st.p.alphabet, 4);
    put_le(out, st.N, 8);
    put_le(out, st.words.size(), 8);
    put_le(out, P, 4);
    put_le(out, table.bytes.size(), 4);
    put_le(out, (uint64_t)P * 4 * (1 + W), 4);
    put_le(out, st.part_size, 4);
    out.insert(out.end(), table.bytes.begin(), table.bytes.end());
    for (uint32_t q = 0; q < P; ++q) {
        put_le(out, st.part_start[q], 4);
        for (uint32_t j = 0; j < W; ++j) put_le(out, st.part_final[(uint64_t)q * W + j], 4);
    }
    for (uint16_t wd : st.words) put_le(out, wd, 2);
    return true;
}

bool write_container(const Stream &st, std::vector<uint8_t> &out) {
    if (st.part_size) return write_partitioned(st, out);
    // One table series, or (adaptive) one per table back to back in one bit stream.
    BitWriter table;
    for (uint32_t t = 0; t < st.tables; ++t) {
        std::vector<int64_t> fv(st.f.begin() + (size_t)t * st.p.alphabet,
                                st.f.begin() + (size_t)(t + 1) * st.p.alphabet);
        if (!put_series(table, fv, 5, false)) return false;
    }
    std::vector<uint8_t> meta;
    if (!write_metadata(st, meta)) return false;
    out.clear();
    out.push_back('R'); out.push_back('C'); out.push_back(st.adaptive ? 'A' : 'L'); out.push_back('1');
    put_le(out, 1, 2);
    out.push_back((uint8_t)st.p.lanes);
    out.push_back((uint8_t)st.p.quant_bits);
    out.push_back((uint8_t)st.p.symbol_bytes);
    out.push_back((uint8_t)st.p.l_bits);
    out.push_back((uint8_t)st.p.b_bits);
    out.push_back(0);
    put_le(out, st.p.alphabet, 4);
    put_le(out, st.N, 8);
    put_le(out, st.words.size(), 8);
    put_le(out, st.threads(), 4);
    put_le(out, table.bytes.size(), 4);
    put_le(out, meta.size(), 4);
    put_le(out, st.adaptive ? st.tables : 0, 4);
    out.insert(out.end(), table.bytes.begin(), table.bytes.end());
    for (uint32_t x : st.final_state) put_le(out, x, 4);
    out.insert(out.end(), meta.begin(), meta.end());
    for (uint16_t wd : st.words) put_le(out, wd, 2);
    return true;
}

int read_partitioned(const uint8_t *c, uint64_t len, Stream &st, orc_info *info) {
    st.p.lanes = c[6];
    st.p.quant_bits = c[7];
    st.p.symbol_bytes = c[8];
    st.p.l_bits = c[9];
    st.p.b_bits = c[10];
    st.p.alphabet = (uint32_t)get_le(c + 12, 4);
    if (!params_ok(st.p)) return ORC_CORRUPT;
    st.N = get_le(c + 16, 8);
    const uint64_t B = get_le(c + 24, 8);
    const uint32_t P = (uint32_t)get_le(c + 32, 4);
    const uint64_t table_bytes = get_le(c + 36, 4);
    const uint64_t meta_bytes = get_le(c + 40, 4);
    const uint64_t S = get_le(c + 44, 4);
    const uint64_t W = st.p.lanes;
    if (S == 0 || S % W != 0 || P != std::max<uint64_t>(1, ceil_div(st.N, S))) return ORC_CORRUPT;
    if (meta_bytes != (uint64_t)P * 4 * (1 + W) || B > len || 48 + table_bytes + meta_bytes + 2 * B != len)
        return ORC_CORRUPT;
    if (info) {
        info->n_symbols = st.N; info->n_words = B; info->threads = P;
        info->lanes = st.p.lanes; info->quant_bits = st.p.quant_bits;
        info->symbol_bytes = st.p.symbol_bytes; info->alphabet = st.p.alphabet;
        info->l_bits = st.p.l_bits; info->b_bits = st.p.b_bits;
        info->table_bytes = table_bytes; info->metadata_bytes = meta_bytes; info->total_bytes = len;
    }
    const uint8_t *q = c + 48;
    BitReader tr{q, table_bytes};
    std::vector<int64_t> fv;
    if (!get_series(tr, st.p.alphabet, 5, false, fv) || ceil_div(tr.pos, 8) != table_bytes) return ORC_CORRUPT;
    uint64_t total = 0;
    st.f.assign(st.p.alphabet, 0);
    for (uint32_t s = 0; s < st.p.alphabet; ++s) { st.f[s] = (uint32_t)fv[s]; total += st.f[s]; }
    if (total != (1ull << st.p.quant_bits)) return ORC_CORRUPT;
    q += table_bytes;
    st.part_size = S;
    st.part_start.resize(P);
    st.part_final.resize((uint64_t)P * W);
    for (uint32_t k = 0; k < P; ++k) {
        st.part_start[k] = get_le(q, 4);
        q += 4;
        for (uint64_t j = 0; j < W; ++j, q += 4) st.part_final[(uint64_t)k * W + j] = (uint32_t)get_le(q, 4);
        if (st.part_start[k] > B || (k > 0 && st.part_start[k] < st.part_start[k - 1])) return ORC_CORRUPT;
    }
    if (P && st.part_start[0] != 0) return ORC_CORRUPT;
    st.splits.clear();
    st.words.resize(B);
    for (uint64_t k = 0; k < B; ++k) st.words[k] = (uint16_t)get_le(q + 2 * k, 2);
    return ORC_OK;
}

int read_container(const uint8_t *c, uint64_t len, Stream &st, orc_info *info) {
    if (len >= 48 && std::memcmp(c, "RCP1", 4) == 0 && get_le(c + 4, 2) == 1) return read_partitioned(c, len, st, info);
    if (len < 48 || get_le(c + 4, 2) != 1) return ORC_CORRUPT;
    st.adaptive = std::memcmp(c, "RCA1", 4) == 0;
    if (!st.adaptive && std::memcmp(c, "RCL1", 4) != 0) return ORC_CORRUPT;
    st.tables = st.adaptive ? (uint32_t)get_le(c + 44, 4) : 1u;
    if (st.tables < 1 || st.tables > 256) return ORC_CORRUPT;
    st.p.lanes = c[6];
    st.p.quant_bits = c[7];
    st.p.symbol_bytes = c[8];
    st.p.l_bits = c[9];
    st.p.b_bits = c[10];
    st.p.alphabet = (uint32_t)get_le(c + 12, 4);
    if (!params_ok(st.p)) return ORC_CORRUPT;
    st.N = get_le(c + 16, 8);
    const uint64_t B = get_le(c + 24, 8);
    const uint32_t M = (uint32_t)get_le(c + 32, 4);
    const uint64_t table_bytes = get_le(c + 36, 4);
    const uint64_t meta_bytes = get_le(c + 40, 4);
    const uint64_t W = st.p.lanes;
    if (M < 1) return ORC_CORRUPT;
    const uint64_t need = 48 + table_bytes + 4 * W + meta_bytes + 2 * B;
    if (B > len || need != len) return ORC_CORRUPT;
    if (info) {
        info->n_symbols = st.N; info->n_words = B; info->threads = M;
        info->lanes = st.p.lanes; info->quant_bits = st.p.quant_bits;
        info->symbol_bytes = st.p.symbol_bytes; info->alphabet = st.p.alphabet;
        info->l_bits = st.p.l_bits; info->b_bits = st.p.b_bits;
        info->table_bytes = table_bytes; info->metadata_bytes = meta_bytes; info->total_bytes = len;
    }
    const uint8_t *q = c + 48;
    BitReader tr{q, table_bytes};
    st.f.assign((size_t)st.tables * st.p.alphabet, 0);
    for (uint32_t t = 0; t < st.tables; ++t) {
        std::vector<int64_t> fv;
        if (!get_series(tr, st.p.alphabet, 5, false, fv)) return ORC_CORRUPT;
        uint64_t total = 0;
        for (uint32_t s = 0; s < st.p.alphabet; ++s) {
            st.f[(size_t)t * st.p.alphabet + s] = (uint32_t)fv[s];
            total += (uint64_t)fv[s];
        }
        if (total != (1ull << st.p.quant_bits)) return ORC_CORRUPT;
    }
    if (ceil_div(tr.pos, 8) != table_bytes) return ORC_CORRUPT;
    q += table_bytes;
    st.final_state.resize(W);
    for (uint64_t j = 0; j < W; ++j) st.final_state[j] = (uint32_t)get_le(q + 4 * j, 4);
    q += 4 * W;
    st.splits.clear();
    if (M > 1) {
        const uint64_t G = ceil_div(st.N, W);
        const uint64_t Eb = ceil_div(B, M), Eg = ceil_div(G, M);
        BitReader r{q, meta_bytes};
        std::vector<int64_t> O, X;
        if (!get_series(r, M - 1, 5, true, O) || !get_series(r, M - 1, 5, true, X)) return ORC_CORRUPT;
        for (uint32_t k = 1; k < M; ++k) {
            Split sp;
            int64_t pos_plus_one = O[k - 1] + (int64_t)(k * Eb);
            int64_t anchor = X[k - 1] + (int64_t)(k * Eg) - 1;   // back to a 0-based group
            if (pos_plus_one < 1 || (uint64_t)pos_plus_one > B || anchor < 0) return ORC_CORRUPT;
            sp.pos = (uint64_t)pos_plus_one - 1;
            sp.state.resize(W);
            for (uint64_t j = 0; j < W; ++j) sp.state[j] = (uint32_t)r.get(16);
            std::vector<int64_t> d;
            if (!get_series(r, W, 4, false, d)) return ORC_CORRUPT;
            sp.index.resize(W);
            int64_t min_d = d[0];
            for (uint64_t j = 0; j < W; ++j) {
                min_d = std::min(min_d, d[j]);
                int64_t g = anchor - d[j];
                if (g < 0) return ORC_CORRUPT;
                sp.index[j] = g * (int64_t)W + (int64_t)j;
                if (sp.state[j] == 0 || sp.state[j] >= (1u << st.p.l_bits)) return ORC_CORRUPT;
            }
            if (min_d != 0 || sp.imax() >= (int64_t)st.N) return ORC_CORRUPT;
            if (!st.splits.empty()) {
                const Split &pv = st.splits.back();
                if (sp.pos <= pv.pos || sp.imin() < pv.imin()) return ORC_CORRUPT;
            }
            st.splits.push_back(std::move(sp));
        }
        if (r.overrun || ceil_div(r.pos, 8) != meta_bytes) return ORC_CORRUPT;
    } else if (meta_bytes != 0) {
        return ORC_CORRUPT;
    }
    q += meta_bytes;
    st.words.resize(B);
    for (uint64_t k = 0; k < B; ++k) st.words[k] = (uint16_t)get_le(q + 2 * k, 2);
    return ORC_OK;
}

// ---------------------------------------------------------------------------
// Decoding
// ---------------------------------------------------------------------------

// Eq. 2 for one lane: returns the symbol and updates x.
uint32_t decode_step(uint64_t &x, const std::vector<uint32_t> &f, const std::vector<uint64_t> &F,
                     uint32_t n) {
    uint64_t slot = x % (1ull << n);
    uint32_t s = 0;
    while (!(F[s] <= slot && slot < F[s + 1])) ++s;     // s = t with F(t) <= x mod 2^n < F(t+1)
    x = (uint64_t)f[s] * (x >> n) - F[s] + slot;
    return s;
}

// One thread of the Recoil decoder (Sec. 4.1). Thread t (1..M) starts at
// split point t, or at the final states for t = M, and walks symbol groups
// downwards. A lane is switched on just before its first read (synchronisation
// phase); symbols are kept only inside [lo, hi).
int decode_thread(const Stream &st, uint32_t t, uint64_t lo, uint64_t hi, void *out,
                  std::vector<int64_t> *trace = nullptr) {
    if (st.adaptive && st.tidx.size() != st.N) return ORC_BAD_PARAM;   // the table index is not set
    const uint32_t W = st.p.lanes, n = st.p.quant_bits, b = st.p.b_bits;
    const uint64_t L = 1ull << st.p.l_bits;
    const uint32_t M = st.threads();
    std::vector<std::vector<uint32_t>> fs;
    std::vector<std::vector<uint64_t>> Fs;
    tables_of(st, fs, Fs);
    std::vector<uint64_t> x(W, 0);
    std::vector<bool> active(W, false);
    std::vector<int64_t> init_group(W, 0);
    int64_t p;              // next word to read
    int64_t top;            // first group decoded
    if (t == M) {
        for (uint32_t j = 0; j < W; ++j) { x[j] = st.final_state[j]; active[j] = true; }
        p = (int64_t)st.words.size() - 1;
        top = (int64_t)st.groups() - 1;
    } else {
        const Split &sp = st.splits[t - 1];
        for (uint32_t j = 0; j < W; ++j) init_group[j] = sp.index[j] / W;
        p = (int64_t)sp.pos;
        top = sp.imax() / W;
    }
    if (lo >= hi) return ORC_OK;
    for (int64_t h = top; h >= 0; --h) {
        // Read step before decoding group h, in decreasing lane order (Sec. 2.2).
        for (int j = (int)W - 1; j >= 0; --j) {
            if (!active[j] && init_group[j] == h) { active[j] = true; x[j] = st.splits[t - 1].state[j]; }
            if (active[j] && x[j] < L) {
                if (p < 0) return ORC_CORRUPT;
                x[j] = (x[j] << b) | st.words[(uint64_t)p];      // Eq. 4
                --p;
            }
        }
        // Decode group h (Eq. 2).
        for (uint32_t j = 0; j < W; ++j) {
            uint64_t i = (uint64_t)h * W + j;
            if (!active[j] || i >= st.N) continue;
            const uint32_t ti = st.table_of(i);
            uint32_t s = decode_step(x[j], fs[ti], Fs[ti], n);
            if (trace) trace->push_back((int64_t)i);
            if (i >= lo && i < hi) store_symbol(out, st.p.symbol_bytes, i, s);
        }
        if ((uint64_t)h * W <= lo) break;   // the group holding lo is done
    }
    return ORC_OK;
}

void thread_range(const Stream &st, uint32_t t, bool aligned, uint64_t &lo, uint64_t &hi) {
    if (st.part_size) {
        lo = (uint64_t)(t - 1) * st.part_size;
        hi = std::min<uint64_t>(st.N, lo + st.part_size);
        return;
    }
    const uint32_t M = st.threads();
    const uint64_t W = st.p.lanes;
    auto imin = [&](uint32_t k) -> uint64_t {   // Imin_0 = 0, Imin_M = N
        if (k == 0) return 0;
        if (k == M) return st.N;
        return (uint64_t)st.splits[k - 1].imin();
    };
    if (!aligned) { lo = imin(t - 1); hi = imin(t); return; }
    // Whole groups: thread t owns groups floor(Imin_{t-1}/W)+1 .. floor(Imin_t/W).
    lo = (t == 1) ? 0 : (imin(t - 1) / W + 1) * W;
    hi = (t == M) ? st.N : std::min<uint64_t>(st.N, (imin(t) / W + 1) * W);
    if (hi < lo) hi = lo;
}

// Sub-sequence q of a conventional container: plain interleaved decoding of its
// own words from its own final states (Eq. 2, Eq. 4), symbols [lo, hi).
int decode_partition(const Stream &st, uint32_t q, void *out) {
    const uint32_t W = st.p.lanes, n = st.p.quant_bits, b = st.p.b_bits;
    const uint64_t L = 1ull << st.p.l_bits;
    const std::vector<uint64_t> F = cdf_of(st.f);
    const uint64_t lo = (uint64_t)q * st.part_size, hi = std::min<uint64_t>(st.N, lo + st.part_size);
    const int64_t first = (int64_t)st.part_start[q];
    const int64_t end = q + 1 < st.threads() ? (int64_t)st.part_start[q + 1] : (int64_t)st.words.size();
    std::vector<uint64_t> x(W);
    for (uint32_t j = 0; j < W; ++j) x[j] = st.part_final[(uint64_t)q * W + j];
    int64_t p = end - 1;
    const int64_t groups = (int64_t)ceil_div(hi - lo, W);
    for (int64_t h = groups - 1; h >= 0; --h) {
        for (uint32_t j = 0; j < W; ++j) {
            uint64_t i = lo + (uint64_t)h * W + j;
            if (i < hi) store_symbol(out, st.p.symbol_bytes, i, decode_step(x[j], st.f, F, n));
        }
        for (int j = (int)W - 1; j >= 0; --j) {
            if (x[j] < L) {
                if (p < first) return ORC_CORRUPT;
                x[j] = (x[j] << b) | st.words[(uint64_t)p];
                --p;
            }
        }
    }
    // Every lane of the sub-sequence started at L and read only its own words.
    if (p != first - 1) return ORC_CORRUPT;
    for (uint32_t j = 0; j < W; ++j) if (x[j] != L) return ORC_CORRUPT;
    return ORC_OK;
}

int decode_serial(const Stream &st, void *out) {
    if (st.part_size) {
        for (uint32_t q = 0; q < st.threads(); ++q) {
            int rc = decode_partition(st, q, out);
            if (rc) return rc;
        }
        return ORC_OK;
    }
    if (st.adaptive && st.tidx.size() != st.N) return ORC_BAD_PARAM;
    const uint32_t W = st.p.lanes, n = st.p.quant_bits, b = st.p.b_bits;
    const uint64_t L = 1ull << st.p.l_bits;
    std::vector<std::vector<uint32_t>> fs;
    std::vector<std::vector<uint64_t>> Fs;
    tables_of(st, fs, Fs);
    std::vector<uint64_t> x(st.final_state.begin(), st.final_state.end());
    int64_t p = (int64_t)st.words.size() - 1;
    for (int64_t h = (int64_t)st.groups() - 1; h >= 0; --h) {
        for (uint32_t j = 0; j < W; ++j) {
            uint64_t i = (uint64_t)h * W + j;
            if (i >= st.N) continue;
            const uint32_t ti = st.table_of(i);
            store_symbol(out, st.p.symbol_bytes, i, decode_step(x[j], fs[ti], Fs[ti], n));
        }
        for (int j = (int)W - 1; j >= 0; --j) {     // read step before group h-1
            if (x[j] < L) {
                if (p < 0) return ORC_CORRUPT;
                x[j] = (x[j] << b) | st.words[(uint64_t)p];
                --p;
            }
        }
    }
    // The encoder started every lane at L and consumed nothing else.
    if (p != -1) return ORC_CORRUPT;
    for (uint32_t j = 0; j < W; ++j) if (x[j] != L) return ORC_CORRUPT;
    return ORC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Encoder
// ---------------------------------------------------------------------------
struct orc_enc {
    Stream st;
    std::vector<int64_t> ev_idx;     // event k wrote word k
    std::vector<uint32_t> ev_state;
    uint64_t n_candidates = 0;
};
struct orc_dec {
    Stream st;
};

extern "C" int orc_quantize(const uint64_t *counts, uint32_t A, uint32_t n, uint32_t *f_out) {
    // Quantisation rule (the paper only says tables come from symbol statistics):
    // f = max(1, floor(c * 2^n / N)) for present symbols; a shortfall is handed
    // out one unit at a time by largest remainder (ties: smaller symbol); an
    // excess is taken one unit at a time from the largest f > 1 (ties: smaller symbol).
    if (n < 1 || n > 16 || A < 1) return ORC_BAD_PARAM;
    const uint64_t total = 1ull << n;
    uint64_t N = 0, present = 0;
    for (uint32_t s = 0; s < A; ++s) { N += counts[s]; present += counts[s] > 0; }
    if (present == 0 || present > total) return ORC_INFEASIBLE;
    std::vector<uint64_t> f(A, 0), rem(A, 0);
    uint64_t sum = 0;
    for (uint32_t s = 0; s < A; ++s) {
        if (!counts[s]) continue;
        unsigned __int128 scaled = (unsigned __int128)counts[s] * total;
        f[s] = (uint64_t)(scaled / N);
        rem[s] = (uint64_t)(scaled % N);
        if (f[s] == 0) f[s] = 1;
        sum += f[s];
    }
    // The floors lose less than one unit per present symbol, so the shortfall
    // is smaller than the number of present symbols: one pass suffices.
    std::vector<bool> given(A, false);
    while (sum < total) {
        int best = -1;
        for (uint32_t s = 0; s < A; ++s) {
            if (!counts[s] || given[s]) continue;
            if (best < 0 || rem[s] > rem[best]) best = (int)s;
        }
        f[best] += 1;
        given[best] = true;
        sum += 1;
    }
    while (sum > total) {
        int best = -1;
        for (uint32_t s = 0; s < A; ++s)
            if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = (int)s;
        f[best] -= 1;
        sum -= 1;
    }
    for (uint32_t s = 0; s < A; ++s) f_out[s] = (uint32_t)f[s];
    return ORC_OK;
}

namespace {

int encode_body(const void *symbols, orc_enc *e, uint32_t threads, orc_enc **out);

// Recoil encoding (Sec. 4). tidx == NULL: one table (given, or quantised from the
// counts). Otherwise adaptive coding: T given tables and symbol i coded with table
// tidx[i] (Sec. 3.1); everything else is the same.
int encode_impl(const void *symbols, uint64_t N, const orc_params *pp, const uint32_t *freq, uint32_t T,
                const uint8_t *tidx, uint32_t threads, orc_enc **out) {
    *out = nullptr;
    if (!pp || !params_ok(*pp) || threads < 1) return ORC_BAD_PARAM;
    if (tidx && (!freq || T < 1 || T > 256)) return ORC_BAD_PARAM;
    const orc_params P = *pp;
    auto *e = new (std::nothrow) orc_enc();
    if (!e) return ORC_BAD_PARAM;
    Stream &st = e->st;
    st.p = P;
    st.N = N;
    for (uint64_t i = 0; i < N; ++i)
        if (symbol_at(symbols, P.symbol_bytes, i) >= P.alphabet || (tidx && tidx[i] >= T)) { delete e; return ORC_BAD_PARAM; }
    if (tidx) {
        st.adaptive = true;
        st.tables = T;
        st.tidx.assign(tidx, tidx + N);
        st.f.assign(freq, freq + (size_t)T * P.alphabet);
        for (uint32_t t = 0; t < T; ++t) {
            uint64_t total = 0;
            for (uint32_t s = 0; s < P.alphabet; ++s) total += st.f[(size_t)t * P.alphabet + s];
            if (total != (1ull << P.quant_bits)) { delete e; return ORC_BAD_PARAM; }
        }
        for (uint64_t i = 0; i < N; ++i)
            if (st.f[(size_t)tidx[i] * P.alphabet + symbol_at(symbols, P.symbol_bytes, i)] == 0) { delete e; return ORC_INFEASIBLE; }
        return encode_body(symbols, e, threads, out);
    }
    // Table: given, or quantised from the symbol counts.
    st.f.assign(P.alphabet, 0);
    if (freq) {
        uint64_t total = 0;
        for (uint32_t s = 0; s < P.alphabet; ++s) { st.f[s] = freq[s]; total += freq[s]; }
        if (total != (1ull << P.quant_bits)) { delete e; return ORC_BAD_PARAM; }
    } else if (N > 0) {
        std::vector<uint64_t> counts(P.alphabet, 0);
        for (uint64_t i = 0; i < N; ++i) counts[symbol_at(symbols, P.symbol_bytes, i)]++;
        int rc = orc_quantize(counts.data(), P.alphabet, P.quant_bits, st.f.data());
        if (rc) { delete e; return rc; }
    } else {
        st.f[0] = 1u << P.quant_bits;
    }
    for (uint64_t i = 0; i < N; ++i)
        if (st.f[symbol_at(symbols, P.symbol_bytes, i)] == 0) { delete e; return ORC_INFEASIBLE; }
    return encode_body(symbols, e, threads, out);
}

}  // namespace

extern "C" int orc_encode(const void *symbols, uint64_t N, const orc_params *pp, const uint32_t *freq,
                          uint32_t threads, orc_enc **out) {
    return encode_impl(symbols, N, pp, freq, 1, nullptr, threads, out);
}

extern "C" int orc_encode_adaptive(const void *symbols, uint64_t N, const orc_params *pp, const uint32_t *freqs,
                                   uint32_t tables, const uint8_t *tidx, uint32_t threads, orc_enc **out) {
    if (!tidx && N > 0) return ORC_BAD_PARAM;
    static const uint8_t none = 0;
    return encode_impl(symbols, N, pp, freqs, tables, tidx ? tidx : &none, threads, out);
}

namespace {

// The encoder proper, once the table(s) are set: interleaved coding, candidate
// scan, split choice and the backward scan of each chosen split.
int encode_body(const void *symbols, orc_enc *e, uint32_t threads, orc_enc **out) {
    Stream &st = e->st;
    const orc_params P = st.p;
    const uint64_t N = st.N;
    std::vector<std::vector<uint32_t>> fs;
    std::vector<std::vector<uint64_t>> Fs;
    tables_of(st, fs, Fs);

    // Interleaved encode (Eq. 1 with the renormalisation of Eq. 3, Sec. 2.2).
    const uint32_t W = P.lanes, n = P.quant_bits, b = P.b_bits;
    const uint64_t L = 1ull << P.l_bits;
    std::vector<uint64_t> x(W, L);                 // initial state: L in every lane
    const uint64_t G = st.groups();
    for (uint64_t g = 0; g < G; ++g) {
        for (uint32_t j = 0; j < W; ++j) {
            uint64_t i = g * W + j;
            if (i >= N) break;
            uint32_t s = symbol_at(symbols, P.symbol_bytes, i);
            const uint32_t ti = st.table_of(i);
            const std::vector<uint64_t> &F = Fs[ti];
            uint64_t fs_ = fs[ti][s];
            // Renormalise against the frequency of the symbol about to be encoded:
            // emit the low b bits, then shift (the paper prints these two
            // assignments in the opposite order).
            if (x[j] >= ((L >> n) << b) * fs_) {
                st.words.push_back((uint16_t)(x[j] & ((1ull << b) - 1)));
                x[j] >>= b;
                e->ev_idx.push_back((int64_t)i - (int64_t)W);   // the lane's previous symbol
                e->ev_state.push_back((uint32_t)x[j]);
            }
            x[j] = ((x[j] / fs_) << n) + F[s] + (x[j] % fs_);   // Eq. 1
        }
    }
    st.final_state.assign(x.begin(), x.end());
    const uint64_t B = st.words.size();

    // Candidate scan (Sec. 4.1): word k is a usable split point when every lane
    // has renormalised at or before it, with a non-negative symbol index and a
    // symbol-group distance to the anchor that fits the 16-bit series.
    std::vector<int64_t> last(W, -1);
    std::vector<uint8_t> valid(B, 0);
    std::vector<int64_t> cand_min(B, 0);
    for (uint64_t k = 0; k < B; ++k) {
        int64_t idx = e->ev_idx[k];
        if (idx >= 0) last[(uint64_t)idx % W] = idx;
        int64_t mn = INT64_MAX, mx = -1;
        for (uint32_t j = 0; j < W; ++j) { mn = std::min(mn, last[j]); mx = std::max(mx, last[j]); }
        if (mn < 0 || idx < 0) continue;
        if ((uint64_t)(mx / W - mn / W) >= 65536) continue;
        valid[k] = 1;
        cand_min[k] = mn;
        e->n_candidates++;
    }

    // Split choice (Def. 4.1), greedy in word order. For split k the target T is
    // recomputed from the symbols that remain; the window ends where
    // t exceeds 2T + t_s; ties go to the earliest word.
    std::vector<uint64_t> chosen;
    int64_t prev_max = -1;
    uint64_t ci = 0;
    for (uint32_t k = 1; k < threads; ++k) {
        const int64_t remaining = (int64_t)N - prev_max - 1;
        const int64_t T = (int64_t)ceil_div((uint64_t)std::max<int64_t>(remaining, 0), threads - k + 1);
        int64_t best = -1, best_h = 0;
        for (; ci < B; ++ci) {
            if (!valid[ci]) continue;
            const int64_t imax = e->ev_idx[ci];
            const int64_t t = imax - prev_max;
            const int64_t ts = imax - cand_min[ci] + 1;
            if (best >= 0 && t > 2 * T + ts) break;
            const int64_t h = std::llabs(t - T) + std::llabs(t - ts - T);
            if (best < 0 || h < best_h) { best = (int64_t)ci; best_h = h; }
            if (t > 2 * T + ts) { ++ci; break; }
        }
        if (best < 0) break;            // no candidates left: fewer threads
        chosen.push_back((uint64_t)best);
        prev_max = e->ev_idx[(uint64_t)best];
        ci = (uint64_t)best + 1;
    }

    // Record each chosen split by a backward scan from its word.
    for (uint64_t pos : chosen) {
        Split sp;
        sp.pos = pos;
        sp.state.assign(W, 0);
        sp.index.assign(W, -1);
        uint32_t seen = 0;
        for (int64_t k = (int64_t)pos; k >= 0 && seen < W; --k) {
            int64_t idx = e->ev_idx[(uint64_t)k];
            if (idx < 0) continue;
            uint32_t j = (uint32_t)((uint64_t)idx % W);
            if (sp.index[j] >= 0) continue;    // only each lane's latest event counts
            sp.index[j] = idx;
            sp.state[j] = e->ev_state[(uint64_t)k];
            ++seen;
        }
        st.splits.push_back(std::move(sp));
    }
    *out = e;
    return ORC_OK;
}

}  // namespace

extern "C" void orc_enc_free(orc_enc *e) { delete e; }

extern "C" int orc_set_table_index(orc_dec *d, const uint8_t *tidx, uint64_t n) {
    if (!d || !d->st.adaptive || n != d->st.N || (n && !tidx)) return ORC_BAD_PARAM;
    for (uint64_t i = 0; i < n; ++i) if (tidx[i] >= d->st.tables) return ORC_BAD_PARAM;
    d->st.tidx.assign(tidx, tidx + n);
    return ORC_OK;
}

// Conventional partitioning (Sec. 2.3), the comparison baseline: the symbol sequence
// is cut into sub-sequences of S symbols (S = ceil(N / P) rounded up to whole groups
// of W, so every sub-sequence but the last has full groups and lane i mod W), each
// coded by its own W interleaved encoders from state L (Eq. 1, Eq. 3) with one table
// for the whole sequence; the sub-bitstreams are concatenated.
extern "C" int orc_encode_partitioned(const void *symbols, uint64_t N, const orc_params *pp, const uint32_t *freq,
                                      uint32_t partitions, uint8_t *dst, uint64_t cap, uint64_t *written) {
    if (!pp || !params_ok(*pp) || partitions < 1 || !written) return ORC_BAD_PARAM;
    const orc_params P = *pp;
    Stream st;
    st.p = P;
    st.N = N;
    st.f.assign(P.alphabet, 0);
    for (uint64_t i = 0; i < N; ++i)
        if (symbol_at(symbols, P.symbol_bytes, i) >= P.alphabet) return ORC_BAD_PARAM;
    if (freq) {
        uint64_t total = 0;
        for (uint32_t s = 0; s < P.alphabet; ++s) { st.f[s] = freq[s]; total += freq[s]; }
        if (total != (1ull << P.quant_bits)) return ORC_BAD_PARAM;
    } else if (N > 0) {
        std::vector<uint64_t> counts(P.alphabet, 0);
        for (uint64_t i = 0; i < N; ++i) counts[symbol_at(symbols, P.symbol_bytes, i)]++;
        int rc = orc_quantize(counts.data(), P.alphabet, P.quant_bits, st.f.data());
        if (rc) return rc;
    } else {
        st.f[0] = 1u << P.quant_bits;
    }
    for (uint64_t i = 0; i < N; ++i)
        if (st.f[symbol_at(symbols, P.symbol_bytes, i)] == 0) return ORC_INFEASIBLE;
    const std::vector<uint64_t> F = cdf_of(st.f);
    const uint32_t W = P.lanes, n = P.quant_bits, b = P.b_bits;
    const uint64_t L = 1ull << P.l_bits;
    const uint64_t S = std::max<uint64_t>(1, ceil_div(std::max<uint64_t>(ceil_div(N, partitions), 1), W)) * W;
    const uint64_t parts = std::max<uint64_t>(1, ceil_div(N, S));
    if (S >= (1ull << 32) || parts >= (1ull << 32)) return ORC_BAD_PARAM;
    st.part_size = S;
    for (uint64_t q = 0; q < parts; ++q) {
        const uint64_t lo = q * S, hi = std::min<uint64_t>(N, lo + S);
        st.part_start.push_back(st.words.size());
        std::vector<uint64_t> x(W, L);
        for (uint64_t i = lo; i < hi; ++i) {
            const uint32_t j = (uint32_t)((i - lo) % W);
            const uint32_t s = symbol_at(symbols, P.symbol_bytes, i);
            const uint64_t fs = st.f[s];
            if (x[j] >= ((L >> n) << b) * fs) {        // renormalise: low b bits out, then shift
                st.words.push_back((uint16_t)(x[j] & ((1ull << b) - 1)));
                x[j] >>= b;
            }
            x[j] = ((x[j] / fs) << n) + F[s] + (x[j] % fs);   // Eq. 1
        }
        for (uint32_t j = 0; j < W; ++j) st.part_final.push_back((uint32_t)x[j]);
        if (st.words.size() >= (1ull << 32)) return ORC_BAD_PARAM;
    }
    std::vector<uint8_t> c;
    if (!write_container(st, c)) return ORC_INFEASIBLE;
    *written = c.size();
    if (!dst) return ORC_OK;
    if (cap < c.size()) return ORC_SMALL_BUFFER;
    std::memcpy(dst, c.data(), c.size());
    return ORC_OK;
}

extern "C" uint64_t orc_enc_container_size(const orc_enc *e) {
    std::vector<uint8_t> c;
    if (!write_container(e->st, c)) return 0;
    return c.size();
}

extern "C" int orc_enc_container(const orc_enc *e, uint8_t *dst, uint64_t cap) {
    std::vector<uint8_t> c;
    if (!write_container(e->st, c)) return ORC_INFEASIBLE;
    if (c.size() > cap) return ORC_SMALL_BUFFER;
    std::memcpy(dst, c.data(), c.size());
    return ORC_OK;
}

extern "C" uint32_t orc_enc_threads(const orc_enc *e) { return e->st.threads(); }
extern "C" uint64_t orc_enc_num_events(const orc_enc *e) { return e->ev_idx.size(); }
extern "C" uint64_t orc_enc_num_candidates(const orc_enc *e) { return e->n_candidates; }

extern "C" int orc_enc_events(const orc_enc *e, orc_event *dst, uint64_t cap) {
    if (cap < e->ev_idx.size()) return ORC_SMALL_BUFFER;
    for (uint64_t k = 0; k < e->ev_idx.size(); ++k) {
        int64_t idx = e->ev_idx[k];
        dst[k].pos = k;
        dst[k].idx = idx;
        dst[k].lane = (uint32_t)(((idx % (int64_t)e->st.p.lanes) + e->st.p.lanes) % e->st.p.lanes);
        dst[k].state = e->ev_state[k];
    }
    return ORC_OK;
}

extern "C" int orc_enc_split(const orc_enc *e, uint32_t k, uint64_t *pos, int64_t *imax, int64_t *imin,
                             uint32_t *states, int64_t *indices) {
    if (k < 1 || k >= e->st.threads()) return ORC_BAD_PARAM;
    const Split &sp = e->st.splits[k - 1];
    *pos = sp.pos; *imax = sp.imax(); *imin = sp.imin();
    for (uint32_t j = 0; j < e->st.p.lanes; ++j) { states[j] = sp.state[j]; indices[j] = sp.index[j]; }
    return ORC_OK;
}

extern "C" int orc_scan_events(const orc_event *ev, uint64_t n_ev, uint32_t W, uint64_t split_event,
                               uint32_t *states, int64_t *indices, int *valid) {
    if (split_event >= n_ev || W < 1) return ORC_BAD_PARAM;
    for (uint32_t j = 0; j < W; ++j) { states[j] = 0; indices[j] = -1; }
    uint32_t seen = 0;
    for (int64_t k = (int64_t)split_event; k >= 0 && seen < W; --k) {
        uint32_t j = ev[k].lane;
        if (j >= W || indices[j] >= 0 || ev[k].idx < 0) continue;
        indices[j] = ev[k].idx;
        states[j] = ev[k].state;
        ++seen;
    }
    *valid = seen == W;
    return ORC_OK;
}

extern "C" int orc_enc_candidate_at(const orc_enc *e, uint64_t pos, int *valid, int64_t *imax,
                                    int64_t *imin, uint32_t *states, int64_t *indices) {
    const uint64_t B = e->ev_idx.size();
    if (pos >= B) return ORC_BAD_PARAM;
    std::vector<orc_event> ev(B);
    orc_enc_events(e, ev.data(), B);
    int rc = orc_scan_events(ev.data(), B, e->st.p.lanes, pos, states, indices, valid);
    if (rc) return rc;
    const uint32_t W = e->st.p.lanes;
    *imax = *std::max_element(indices, indices + W);
    *imin = *std::min_element(indices, indices + W);
    *valid = *valid && e->ev_idx[pos] >= 0 && *imax == e->ev_idx[pos];
    return ORC_OK;
}

extern "C" int orc_series_pack(const int64_t *values, uint64_t count, uint32_t width_field, int is_signed,
                               uint8_t *dst, uint64_t cap, uint64_t *n_bits) {
    BitWriter w;
    std::vector<int64_t> v(values, values + count);
    if (!put_series(w, v, width_field, is_signed != 0)) return ORC_INFEASIBLE;
    if (w.bytes.size() > cap) return ORC_SMALL_BUFFER;
    std::memcpy(dst, w.bytes.data(), w.bytes.size());
    *n_bits = w.nbits;
    return ORC_OK;
}

extern "C" int orc_series_unpack(const uint8_t *src, uint64_t n_bytes, uint64_t count, uint32_t width_field,
                                 int is_signed, int64_t *values, uint64_t *n_bits) {
    BitReader r{src, n_bytes};
    std::vector<int64_t> v;
    if (!get_series(r, count, width_field, is_signed != 0, v)) return ORC_CORRUPT;
    for (uint64_t k = 0; k < count; ++k) values[k] = v[k];
    *n_bits = r.pos;
    return ORC_OK;
}

extern "C" int orc_assemble(const orc_params *p, uint64_t N, const uint32_t *freq, const uint16_t *words,
                            uint64_t B, const uint32_t *final_states, uint32_t threads,
                            const uint64_t *split_pos, const uint32_t *split_states,
                            const int64_t *split_indices, uint8_t *dst, uint64_t cap, uint64_t *written) {
    if (!p || !params_ok(*p) || threads < 1) return ORC_BAD_PARAM;
    Stream st;
    st.p = *p;
    st.N = N;
    st.f.assign(freq, freq + p->alphabet);
    st.words.assign(words, words + B);
    st.final_state.assign(final_states, final_states + p->lanes);
    for (uint32_t k = 1; k < threads; ++k) {
        Split sp;
        sp.pos = split_pos[k - 1];
        sp.state.assign(split_states + (uint64_t)(k - 1) * p->lanes, split_states + (uint64_t)k * p->lanes);
        sp.index.assign(split_indices + (uint64_t)(k - 1) * p->lanes, split_indices + (uint64_t)k * p->lanes);
        st.splits.push_back(std::move(sp));
    }
    std::vector<uint8_t> outc;
    if (!write_container(st, outc)) return ORC_INFEASIBLE;
    *written = outc.size();
    if (outc.size() > cap) return ORC_SMALL_BUFFER;
    std::memcpy(dst, outc.data(), outc.size());
    return ORC_OK;
}

extern "C" int orc_info_of(const uint8_t *c, uint64_t len, orc_info *out) {
    Stream st;
    return read_container(c, len, st, out);
}

extern "C" int orc_combine(const uint8_t *c, uint64_t len, uint32_t target, uint8_t *dst, uint64_t cap,
                           uint64_t *written) {
    // Sec. 3.3: dropping split metadata merges neighbouring threads; keep every
    // ceil(M_in / M_out)-th split point. The bitstream is untouched.
    Stream st;
    int rc = read_container(c, len, st, nullptr);
    if (rc) return rc;
    if (target < 1 || st.part_size) return ORC_BAD_PARAM;   // sub-sequences cannot be merged (Sec. 2.3)
    const uint32_t M_in = st.threads();
    const uint32_t step = (uint32_t)ceil_div(M_in, std::min(target, M_in));
    std::vector<Split> kept;
    for (uint32_t k = 1; k < M_in; ++k)
        if (k % step == 0) kept.push_back(st.splits[k - 1]);
    st.splits = kept;
    std::vector<uint8_t> outc;
    if (!write_container(st, outc)) return ORC_INFEASIBLE;
    *written = outc.size();
    if (outc.size() > cap) return ORC_SMALL_BUFFER;
    std::memcpy(dst, outc.data(), outc.size());
    return ORC_OK;
}

extern "C" int orc_open(const uint8_t *c, uint64_t len, orc_dec **out) {
    auto *d = new (std::nothrow) orc_dec();
    if (!d) return ORC_BAD_PARAM;
    int rc = read_container(c, len, d->st, nullptr);
    if (rc) { delete d; *out = nullptr; return rc; }
    *out = d;
    return ORC_OK;
}

extern "C" void orc_close(orc_dec *d) { delete d; }

extern "C" int orc_decode_serial(const orc_dec *d, void *out) { return decode_serial(d->st, out); }

extern "C" int orc_thread_range(const orc_dec *d, uint32_t t, int aligned, uint64_t *lo, uint64_t *hi) {
    if (t < 1 || t > d->st.threads()) return ORC_BAD_PARAM;
    thread_range(d->st, t, aligned != 0, *lo, *hi);
    return ORC_OK;
}

extern "C" int orc_decode_thread(const orc_dec *d, uint32_t t, int aligned, void *out) {
    if (t < 1 || t > d->st.threads()) return ORC_BAD_PARAM;
    if (d->st.part_size) return decode_partition(d->st, t - 1, out);
    uint64_t lo, hi;
    thread_range(d->st, t, aligned != 0, lo, hi);
    return decode_thread(d->st, t, lo, hi, out);
}

extern "C" int orc_decode_thread_trace(const orc_dec *d, uint32_t t, int aligned, void *out,
                                      int64_t *decoded, uint64_t cap, uint64_t *count) {
    if (t < 1 || t > d->st.threads() || d->st.part_size) return ORC_BAD_PARAM;
    uint64_t lo, hi;
    thread_range(d->st, t, aligned != 0, lo, hi);
    std::vector<int64_t> trace;
    int rc = decode_thread(d->st, t, lo, hi, out, &trace);
    *count = trace.size();
    for (uint64_t k = 0; k < trace.size() && k < cap; ++k) decoded[k] = trace[k];
    return rc;
}

extern "C" int orc_decode_all(const orc_dec *d, int aligned, uint32_t workers, void *out) {
    const uint32_t M = d->st.threads();
    if (workers < 1) workers = 1;
    std::vector<int> rcs(workers, ORC_OK);
    auto run = [&](uint32_t w) {
        // Static contiguous blocks of threads per worker.
        uint32_t a = (uint32_t)((uint64_t)M * w / workers) + 1;
        uint32_t z = (uint32_t)((uint64_t)M * (w + 1) / workers);
        for (uint32_t t = a; t <= z; ++t) {
            int rc = orc_decode_thread(d, t, aligned, out);
            if (rc) { rcs[w] = rc; return; }
        }
    };
    if (workers == 1) {
        run(0);
    } else {
        std::vector<std::thread> pool;
        for (uint32_t w = 0; w < workers; ++w) pool.emplace_back(run, w);
        for (auto &th : pool) th.join();
    }
    for (int rc : rcs) if (rc) return rc;
    return ORC_OK;
}
