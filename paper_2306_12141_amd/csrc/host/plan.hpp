// Host-side GPU decode plan of one stream (shared by single-stream, batched
// and serving paths).
#pragma once

#include <memory>
#include <vector>

#include "../device/decode.hpp"
#include "blob.hpp"

namespace recoil {

struct PlanData {
    std::shared_ptr<const BlobData> blob;
    std::vector<UnitMeta> meta;          // M
    std::vector<uint32_t> lanes;         // M x W
    std::vector<uint8_t> lut;            // 2^n entries, 4 or 8 bytes each
    DecodeTuning tuning;                 // launch shape for recoil_decode
    bool single_symbol = false;
    uint32_t fill_symbol = 0;
    uint32_t units = 0;                  // decode units (meta.size() unless packed)
    // Packed plans: the records are unpacked on the device from the stream's packed
    // metadata section (kept split points (u+1) step, Sec. 3.3); meta and lanes stay empty.
    bool packed = false;
    uint32_t step = 1;
    std::vector<uint8_t> packed_bits;    // the section + 8 zero bytes (the unpacker reads 5-byte windows)
    std::vector<uint32_t> block_bit;     // M - 1 block bit offsets
    // Workspace layout of a single-stream plan (byte offsets from the workspace base).
    size_t off_words = 0, off_lut = 0, off_meta = 0, off_lanes = 0, total = 0;
    size_t off_bits = 0, off_blocks = 0, off_final = 0;   // packed plans
};

constexpr size_t kWsAlign = 256;
// Adaptive coding: the decode tables of all tables must fit LDS beside the rings.
constexpr uint64_t kMaxAdaptiveTableBytes = 65536;
// Wide tables (n > 12): symbols with f > 0, at 8 bytes each beside 16 KiB of buckets.
constexpr uint32_t kMaxWideRanks = 4096;
// Symbols with f > 0 (the entries of a wide table).
uint32_t wide_ranks(const BlobData &b);
// Groups per super-step of the default launch shape: 8 for uint8 tables of n <= 12
// (two 16-wave workgroups per CU still fit LDS), else 4.
inline uint32_t default_chunk_groups(const BlobData &b) {
    return b.symbol_bytes == 1 && !b.adaptive && b.quant_bits <= 12 ? 8u : 4u;
}
inline size_t ws_align(size_t v) { return (v + kWsAlign - 1) / kWsAlign * kWsAlign; }

// Unpack split metadata and build the decode table; fills the single-stream layout.
recoil_status build_plan(const std::shared_ptr<const BlobData> &blob, PlanData &plan);
// The same without unpacking: the decode table and the layout of a plan whose
// records the device unpacks from the packed section, keeping every step-th
// split point for ceil(M / target) units (target 0 or >= M: all).
recoil_status build_plan_packed(const std::shared_ptr<const BlobData> &blob, uint32_t target, PlanData &plan);
// GPU limits on a stream (lanes, n, sizes, adaptive tables); RECOIL_OK if decodable.
recoil_status check_gpu_limits(const BlobData &blob);
// The two halves of build_plan: per-unit and per-lane records only (checks the
// GPU limits and sets the default tuning), and the decode table only.
recoil_status build_units(const std::shared_ptr<const BlobData> &blob, PlanData &plan);
void build_table(const BlobData &blob, PlanData &plan);
// Per-unit records of the blob that combining `blob` to `target` units would
// give, without building that blob; *packed_bytes: its packed metadata size.
recoil_status build_units_combined(const std::shared_ptr<const BlobData> &blob, uint32_t target, PlanData &plan,
                                   uint64_t *packed_bytes);

// Host-to-device copy of pageable host memory: through two pinned staging
// buffers of the calling thread, so it runs at DMA speed. The copies are queued
// on `stream` in order; the call returns once the last one is queued (a staging
// buffer is reused only after its previous copy has completed).
hipError_t stage_h2d(void *dst, const void *src, size_t bytes, hipStream_t stream);

// Bytes of the words section for B words (padded so chunks can be fetched whole).
inline size_t words_section_bytes(uint64_t n_words) { return ws_align(2 * (n_words + kChunkPadWords)); }

}  // namespace recoil
