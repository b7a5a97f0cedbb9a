// Internal host-side types of librecoil.
#pragma once

#include <cstdint>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "recoil.h"

namespace recoil {

// Parameters fixed by the recommended set (Table "rANS parameters"): 32-bit
// states, L = 2^16, 16-bit renormalisation words.
constexpr uint32_t kLowerBits = 16;
constexpr uint32_t kWordBits = 16;
constexpr uint32_t kLower = 1u << kLowerBits;
// The per-lane group distance to the anchor is stored in at most 16 bits (Sec. 4.3).
constexpr uint64_t kMaxGroupDiff = 65535;

// One encoded stream plus its split points, unpacked.
struct BlobData {
    uint32_t lanes = 0, quant_bits = 0, symbol_bytes = 0, alphabet = 0;
    uint64_t n_symbols = 0;
    std::vector<uint32_t> freq;          // f[s], sums to 2^n; adaptive: tables x A, table t at t A
    // Adaptive coding (Sec. 3.1): symbol i was coded with table tidx[i] of `tables`;
    // the index array is side information the decoder is given again.
    bool adaptive = false;
    uint32_t tables = 1;
    std::vector<uint32_t> final_states;  // W
    // B words, written forward, read backward; shared between a blob and the
    // blobs combined from it (the bitstream is the same, only split points differ).
    std::shared_ptr<std::vector<uint16_t>> words_buf = std::make_shared<std::vector<uint16_t>>();
    // Split points k = 1..M-1 (index k-1), increasing word position.
    std::vector<uint64_t> sp_next;       // p_k + 1: words available to the unit starting there
    std::vector<uint64_t> sp_anchor;     // g_k: largest symbol group among the recorded lanes (0-based)
    std::vector<uint16_t> sp_state;      // (M-1) x W recorded post-shift states (< 2^16, Lemma 3.1)
    std::vector<uint16_t> sp_gdiff;      // (M-1) x W: g_k - group of lane j's recorded symbol
    // Conventional partitioning (Sec. 2.3) instead of split points when part_size > 0:
    // sub-sequence q holds symbols [q S, min((q + 1) S, N)) (S = part_size, whole
    // groups of W), coded on its own from state L; its words start at part_start[q]
    // and its final states are part_final[q W .. q W + W - 1].
    uint64_t part_size = 0;
    std::vector<uint64_t> part_start;
    std::vector<uint32_t> part_final;
    // Packed sections, computed once; for the metadata also the bit position of
    // the group series and of each split point's block (so a device can unpack the
    // blocks in parallel).
    std::vector<uint8_t> table_bits;
    std::vector<uint8_t> meta_bits;
    uint64_t x_series_bit = 0;
    std::vector<uint64_t> block_bit;     // M-1

    bool partitioned() const { return part_size != 0; }
    uint32_t splits() const { return partitioned() ? (uint32_t)part_start.size() : (uint32_t)sp_next.size() + 1; }
    uint64_t groups() const { return (n_symbols + lanes - 1) / lanes; }
    const uint16_t *words() const { return words_buf->data(); }
    uint64_t n_words() const { return words_buf->size(); }
    uint64_t total_bytes() const {
        return 48 + table_bits.size() + (partitioned() ? 0 : 4ull * lanes) + meta_bits.size() + 2ull * n_words();
    }
    // Symbol index recorded for lane j at split point k (1-based k).
    uint64_t split_index(uint32_t k, uint32_t j) const {
        uint64_t g = sp_anchor[k - 1] - sp_gdiff[(uint64_t)(k - 1) * lanes + j];
        return g * lanes + j;
    }
};

// Fill table_bits / meta_bits; false if a value does not fit its series.
bool pack_sections(BlobData &b);
// Keep every ceil(M / target)-th split point (Sec. 3.3); the bitstream is shared,
// not copied. nullptr if the re-packed metadata does not fit its series.
std::shared_ptr<BlobData> combine_data(const BlobData &a, uint32_t target);

void set_error(const std::string &msg);
recoil_status fail(recoil_status s, const std::string &msg);

// Runs an entry point's body: host allocation or thread-creation failures inside it
// come back as RECOIL_ERR_OUT_OF_MEMORY instead of crossing the C boundary.
template <typename F>
recoil_status guarded(const char *what, F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(RECOIL_ERR_OUT_OF_MEMORY, std::string(what) + ": out of host memory");
    } catch (const std::exception &e) {
        return fail(RECOIL_ERR_OUT_OF_MEMORY, std::string(what) + ": " + e.what());
    } catch (...) {
        return fail(RECOIL_ERR_OUT_OF_MEMORY, std::string(what) + ": host resources exhausted");
    }
}

}  // namespace recoil

struct recoil_blob {
    std::shared_ptr<const recoil::BlobData> data;
};
