/*
 * librecoil -- parallel rANS decoding with decoder-adaptive scalability on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Lin et al., "Recoil: Parallel rANS Decoding with Decoder-Adaptive
 * Scalability", ICPP 2023. One interleaved rANS bitstream is encoded once; split
 * points are recorded as metadata (per-lane 16-bit intermediate states taken at
 * renormalisation points, plus their symbol indices); the metadata can later be
 * cut down to any smaller number of splits without touching the bitstream; the
 * decoder starts one independent decode unit per split.
 *
 * Terminology used throughout this header:
 *   N        number of symbols; symbols are uint8 or uint16
 *   W        interleaved lanes (32 or 64 on the GPU)
 *   n        quantisation bits: the frequency table f sums to 2^n (Def. 2.1)
 *   L, b     renormalisation lower bound 2^16 and word size 16 bits (Table "rANS parameters")
 *   B        number of 16-bit words in the bitstream
 *   M        number of decode units ("splits"); M - 1 split points are stored
 *   group    symbols gW .. gW+W-1; symbol i belongs to lane i mod W
 *
 * Ownership: host objects (blobs, plans, batches, servers) are created and
 * freed by the library. All device memory is owned by the caller and passed in
 * as plain device pointers; decode calls never allocate, never synchronise and
 * only enqueue work on the given HIP stream.
 *
 * Errors: every call returns a recoil_status (0 = success, < 0 = error);
 * recoil_last_error() returns a thread-local message for the last failure.
 * Corruption that can only be detected while decoding on the device is
 * reported through a caller-owned uint32 error word (see recoil_decode).
 *
 * Container byte layout ("RCL1", little-endian; produced by recoil_blob_serialize):
 *   0  char[4] magic "RCL1"        4  u16 version (1)
 *   6  u8 W                        7  u8 n
 *   8  u8 symbol bytes (1|2)       9  u8 log2 L (16)     10 u8 b (16)   11 u8 0
 *   12 u32 alphabet size A         16 u64 N              24 u64 B
 *   32 u32 M                       36 u32 table bytes    40 u32 metadata bytes  44 u32 0
 *   48 table: f[0..A) as an unsigned bit series with a 5-bit width field
 *      final states: W x u32 (the encoder's last states, transmitted explicitly, Sec. 3.1)
 *      metadata (Sec. 4.3), one MSB-first bit stream, zero-padded to a byte:
 *        signed series (5-bit width field) of (p_k + 1) - k * ceil(B/M), k = 1..M-1
 *        signed series (5-bit width field) of (g_k + 1) - k * ceil(G/M)
 *        per split point k: W x 16-bit states, then an unsigned series
 *        (4-bit width field) of g_k - (group of lane j's recorded symbol)
 *      words: B x u16
 *   where p_k is the word position of split point k, g_k its largest symbol
 *   group (the anchor, 0-based) and G = ceil(N/W). A bit series is a
 *   (width - 1) field followed by one value of `width` bits per element (signed
 *   series put a sign bit before each magnitude); width = max(1, bit length of
 *   the largest magnitude).
 *
 * Adaptive container ("RCA1", recoil_encode_adaptive): the Recoil layout above
 * with magic "RCA1", the number of tables T at offset 44, and a table section
 * holding T series one after another (table t's f[0..A) in the t-th).
 *
 * Conventional partitioned container ("RCP1", the comparison baseline of Sec. 2.3;
 * recoil_encode_partitioned): the same 48-byte header with magic "RCP1", the
 * number of sub-sequences P at offset 32 and the sub-sequence length S (symbols,
 * a multiple of W) at offset 44; then the table; then per sub-sequence q its
 * first word (u32) and its W final states (u32 each); then the B words of all
 * sub-sequences, concatenated. Sub-sequence q holds symbols [q S, min((q+1) S, N)).
 */
#ifndef RECOIL_H
#define RECOIL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t recoil_status;
enum {
    RECOIL_OK = 0,
    RECOIL_ERR_INVALID_ARG = -1,    /* a NULL pointer, a size or a parameter out of range */
    RECOIL_ERR_INFEASIBLE = -2,     /* more distinct symbols than 2^n, or metadata that does not fit */
    RECOIL_ERR_CORRUPT = -3,        /* container failed validation */
    RECOIL_ERR_UNSUPPORTED = -4,    /* valid container outside what the GPU decoder handles */
    RECOIL_ERR_BUFFER_TOO_SMALL = -5,
    RECOIL_ERR_HIP = -6,            /* a HIP runtime call failed */
    RECOIL_ERR_ALIGNMENT = -7,      /* a device pointer is not aligned as required */
    RECOIL_ERR_BUSY = -8,           /* serving: request refused by admission control */
    RECOIL_ERR_NOT_FOUND = -9,
    RECOIL_ERR_OUT_OF_MEMORY = -10, /* host memory or threads could not be obtained */
};

/* Device error word bits (set with atomic OR by the decode kernels). */
enum {
    RECOIL_DEVERR_UNDERFLOW = 1u,   /* a decode unit ran out of bitstream words */
    RECOIL_DEVERR_BAD_ITEM = 2u,    /* batched decode: malformed work item */
};

typedef struct {
    uint32_t lanes;         /* W: 32 or 64 for GPU decoding (1..64 accepted by the encoder) */
    uint32_t quant_bits;    /* n: 1..16 accepted by the encoder; GPU decoding needs 8 <= n <= 16 (n > 12:
                               single-stream decode, at most 4096 symbols with f > 0, not adaptive) */
    uint32_t symbol_bytes;  /* 1 (uint8) or 2 (uint16) */
    uint32_t alphabet;      /* A: symbols lie in [0, A); A <= 256 for uint8, <= 65536 for uint16 */
} recoil_config;

typedef struct {
    uint64_t n_symbols;      /* N */
    uint64_t n_words;        /* B */
    uint32_t splits;         /* M */
    uint32_t lanes, quant_bits, symbol_bytes, alphabet;
    uint64_t table_bytes;    /* packed frequency table */
    uint64_t metadata_bytes; /* packed split metadata (Sec. 4.3) */
    uint64_t total_bytes;    /* whole container: header + table + final states + metadata + words */
} recoil_blob_info_t;

/* Launch shape of the decode kernels.
 *   waves          waves per workgroup (8 or 16); the waves of a workgroup share one
 *                  decode table in LDS. Single-stream decode also takes 1, and 0:
 *                  16, or 1 when the decode has no more wave-sized pieces of work
 *                  (runs, or run pairs for W = 32) than the chip has SIMDs, or 8
 *                  when 16-wave workgroups would not reach every CU, so that the
 *                  waves spread over all CUs
 *   chunk_groups   K (4 or 8): symbol groups per super-step; each unit's LDS bitstream
 *                  ring holds 4 K W words (3 K W ring + K W mirror)
 *   pairs_per_wave batched decode only: work-item size in unit pairs per wave (1..64)
 *   blocks_per_cu  cap on resident workgroups per CU (0: occupancy limit)
 *   units_per_run  k consecutive decode units are decoded as one, from the highest
 *                  unit's split point down to the lowest unit's last group (the decoder
 *                  uses every k-th split point, as combining the splits would, Sec. 3.3,
 *                  without re-packing). 1: every split point. Single-stream decode, 0:
 *                  chosen at launch, ceil(M / resident unit slots), i.e. at most one run
 *                  per unit slot (a wave holds 1 unit, or 2 for W = 32). Batched decode
 *                  (at most 64; 0 is 1): every stream's run length, shortened to
 *                  ceil(M / (waves x units per wave)) for a stream whose M units would
 *                  otherwise leave waves of its workgroup without a run. */
typedef struct {
    uint32_t waves, chunk_groups, pairs_per_wave, blocks_per_cu, units_per_run;
} recoil_tuning;

/* Grid of a single-stream decode and the runs it decodes (recoil_plan_shape).
 * waves_per_block: 1, 8 or 16 (the tuning's, or the one chosen at launch).
 * units_per_wave: runs decoded side by side in one wave: 1 for W = 64; for W = 32,
 * 2 (one per half-wave), or 1 when every run has a wave of its own. */
typedef struct {
    uint32_t blocks, waves_per_block, units_per_run, runs, units_per_wave;
} recoil_decode_shape;

typedef struct recoil_blob recoil_blob;   /* immutable encoded stream; safe to share between threads */
typedef struct recoil_plan recoil_plan;   /* host-side decode plan for one blob on the GPU */

const char *recoil_status_string(recoil_status s);
const char *recoil_last_error(void);
const char *recoil_version(void);

/*
 * Quantise symbol counts to a frequency table summing to 2^n (the paper builds
 * static tables from symbol statistics, Sec. 5.1). Rule: f = max(1, floor(c 2^n / total))
 * for present symbols, 0 otherwise; a shortfall is given out one unit per
 * symbol in order of largest remainder (ties: smaller symbol); an excess is
 * removed one unit at a time from the largest f > 1 (ties: smaller symbol).
 * counts: host array of A uint64; f_out: host array of A uint32.
 * Errors: INVALID_ARG, INFEASIBLE (no symbol present or more than 2^n present).
 */
recoil_status recoil_quantize(const uint64_t *counts, uint32_t alphabet, uint32_t quant_bits,
                              uint32_t *f_out);

/*
 * Encode N symbols with one group of W interleaved rANS coders (Eq. 1 and the
 * renormalisation of Eq. 3; words are appended in increasing lane order within
 * each group, Sec. 2.2) and choose up to n_splits - 1 split points with the
 * heuristic of Def. 4.1, recording for each the states and symbol indices
 * found by the backward scan of Sec. 4.1.
 *
 * symbols: host array of N uint8 or uint16 (per cfg->symbol_bytes), each < A.
 * freq:    host array of A uint32 summing to 2^n, or NULL to quantise the
 *          symbol counts with recoil_quantize.
 * n_splits: requested M >= 1. Fewer units are produced when the stream has
 *          too few usable split points (e.g. N < W gives M = 1).
 * out:     receives a new blob; free with recoil_blob_free.
 * Serial on one host thread (Sec. 6 accepts a slow encoder). Not a hot path.
 * Errors: INVALID_ARG, INFEASIBLE.
 */
recoil_status recoil_encode(const void *symbols, uint64_t n_symbols, const recoil_config *cfg,
                            const uint32_t *freq, uint32_t n_splits, recoil_blob **out);

/*
 * Adaptive coding (Sec. 3.1: the stored symbol indices let each decode unit use a
 * different distribution for every symbol, keyed by its index). Like
 * recoil_encode, but symbol i is coded with table table_index[i] of `tables`
 * tables (freqs: tables x A uint32, table t at t A, each summing to 2^n), in the
 * renormalisation test and in Eq. 1. The index array is side information the
 * decoder already holds (as hyperprior-based image codecs derive it); it is not
 * stored in the container (layout "RCA1" above) and recoil_decode_adaptive takes
 * it again. Split choice, metadata and combining are those of recoil_encode.
 * The GPU decodes uint8 symbols with tables x 2^n x 4 <= 64 KiB.
 * Errors: INVALID_ARG (a table not summing to 2^n, an index >= tables, tables
 * outside 1..256), INFEASIBLE (a symbol with zero frequency in its table).
 */
recoil_status recoil_encode_adaptive(const void *symbols, uint64_t n_symbols, const recoil_config *cfg,
                                     const uint32_t *freqs, uint32_t tables, const uint8_t *table_index,
                                     uint32_t n_splits, recoil_blob **out);

/*
 * The conventional "partitioning symbols" baseline (Sec. 2.3), for comparison:
 * the N symbols are cut into sub-sequences of S = ceil(N / partitions) symbols
 * rounded up to whole groups of W (so fewer sub-sequences when that covers N),
 * each encoded on its own by W interleaved coders from state L with the one
 * table (given, or quantised from the counts of all N symbols), and the
 * sub-bitstreams are concatenated behind an offset table ("RCP1" above). The
 * resulting blob plans and decodes like a Recoil blob (every unit starts from
 * its sub-sequence's final states; there is no synchronisation phase) but its
 * units cannot be combined (recoil_combine_splits returns UNSUPPORTED).
 * Errors: INVALID_ARG, INFEASIBLE, UNSUPPORTED (S, P or B not below 2^32).
 */
recoil_status recoil_encode_partitioned(const void *symbols, uint64_t n_symbols, const recoil_config *cfg,
                                        const uint32_t *freq, uint32_t partitions, recoil_blob **out);

/*
 * Split selection of the encoders (Sec. 4.1, Def. 4.1): threads = 1 uses the
 * streaming chooser inside the encoder's pass; threads >= 2 has the encoder keep a
 * log of its renormalisation events (6 bytes per word) and chooses afterwards with
 * that many threads (a segmented per-lane latest-event scan over word chunks, then
 * the greedy choice over the words in order); 0 (the default) picks the threaded
 * form for streams of 2^24 symbols or more. Every setting chooses the same split
 * points, so the containers are byte-identical. Process-wide; takes effect for
 * encodes started after the call.
 */
void recoil_set_split_writer_threads(uint32_t threads);

/*
 * Decoder-adaptive combining (Sec. 3.3, end of Sec. 4.2): keep every
 * ceil(M_in / target)-th split point, which leaves ceil(M_in / step) decode
 * units (exactly `target` when it divides M_in), and re-express the stored
 * differences against the new expectations. The bitstream is not touched.
 * target >= M_in returns an equal copy. out: new blob.
 * Errors: INVALID_ARG, UNSUPPORTED (a partitioned blob).
 */
recoil_status recoil_combine_splits(const recoil_blob *in, uint32_t target_splits, recoil_blob **out);

/* Container bytes (layout above). Pass dst = NULL to query the size in *written.
 * Errors: INVALID_ARG, BUFFER_TOO_SMALL. */
recoil_status recoil_blob_serialize(const recoil_blob *blob, void *dst, size_t cap, size_t *written);
/* Parse and fully validate a container (header, table, every split point).
 * Errors: INVALID_ARG, CORRUPT. */
recoil_status recoil_blob_deserialize(const void *src, size_t len, recoil_blob **out);
recoil_status recoil_blob_info(const recoil_blob *blob, recoil_blob_info_t *out);
void recoil_blob_free(recoil_blob *blob);

/*
 * Plan a GPU decode of one blob. The plan unpacks the split metadata into a
 * device-friendly layout and reports the device workspace it needs. The plan
 * keeps its own reference to the blob's data; the blob may be freed first.
 * device_bytes: receives the workspace size (bytes, 256-byte aligned sections).
 * For 13 <= n <= 16 (Table 3 allows n <= 16 with b = 16) the decode table has two
 * levels so that it fits LDS: 16-slot buckets, then one entry per symbol with f > 0.
 * Errors: INVALID_ARG, UNSUPPORTED (W not 32/64, n outside 8..16, N or B >= 2^32;
 * n > 12 with more than 4096 symbols of f > 0 or with adaptive tables).
 */
recoil_status recoil_plan_create(const recoil_blob *blob, recoil_plan **out, size_t *device_bytes);
/* Copy bitstream, decode table and unpacked metadata into the caller-owned
 * workspace d_workspace (device pointer, 256-byte aligned, >= device_bytes)
 * with asynchronous copies on `stream`. Host sources stay owned by the plan.
 * Errors: INVALID_ARG, ALIGNMENT, HIP. */
recoil_status recoil_plan_upload(const recoil_plan *plan, void *d_workspace, size_t bytes,
                                 hipStream_t stream);
/* Size in bytes of the split metadata as uploaded (part of device_bytes): unit
 * and lane records, or for a packed plan the packed section, the block offsets
 * and the final states. */
size_t recoil_plan_metadata_device_bytes(const recoil_plan *plan);

/*
 * Device-side metadata unpacking (Sec. 4.3 format). Like recoil_plan_create, but
 * the per-unit and per-lane records are not built on the host: recoil_plan_upload
 * copies the packed metadata section as the container stores it (two signed
 * series, then per split point W 16-bit states and a group-difference series),
 * the bit offset of each split point's block (u32) and the W final states, and
 * queues a kernel on the same stream that writes the records into the workspace
 * before any decode queued after it on that stream.
 * target_units: decode units of the plan; every ceil(M / target)-th split point is
 * kept (the combining of Sec. 3.3, records identical to those of the combined
 * blob; 0 or >= M keeps all M units).
 * recoil_plan_units reports the count only (the records exist on the device);
 * recoil_plan_get_layout gives where they are.
 * Errors: INVALID_ARG, UNSUPPORTED (as recoil_plan_create; conventional
 * partitioned streams; a metadata section of 2^32 bits or more).
 */
recoil_status recoil_plan_create_packed(const recoil_blob *blob, uint32_t target_units, recoil_plan **out,
                                        size_t *device_bytes);
/* Queue only the unpack kernel of a packed plan on `stream`, reading the packed
 * section, block offsets and final states that recoil_plan_upload already placed
 * in d_workspace (which must not have been modified since) and rewriting the
 * unit and lane records. Errors: INVALID_ARG (not a packed plan), ALIGNMENT, HIP. */
recoil_status recoil_plan_unpack(const recoil_plan *plan, void *d_workspace, hipStream_t stream);

/* Byte offsets of a plan's workspace sections (from the workspace base): words,
 * decode table, unit records (unit_count x 4 u32: next, top, ghi, glo, as
 * recoil_plan_units describes) and lane words (unit_count x lanes_per_unit u32:
 * a split point's lane state in bits 0..15 and its activation step in bits
 * 16..31, or the 32-bit final state for the last unit); total = device_bytes. */
typedef struct {
    size_t words, table, units, lanes, total;
    uint32_t unit_count, lanes_per_unit, packed;
} recoil_plan_layout;
recoil_status recoil_plan_get_layout(const recoil_plan *plan, recoil_plan_layout *out);

/* The decode table as uploaded (Eq. 2 per slot): for n <= 12, 2^n entries of 4
 * bytes (uint8: symbol | f << 8 | (slot - F) << 20) or 8 bytes (uint16:
 * f | (slot - F) << 16, symbol), tables x 2^n of them for adaptive streams; for
 * 13 <= n <= 16, 2^(n-4) bucket words (bits 16..31: rank of the symbol holding the
 * bucket's first slot; bit i-1: a symbol's range starts at the bucket's slot i,
 * i = 1..15) and then per symbol with f > 0, in symbol order, the pair (f,
 * symbol | F << 16); zero-padded to 16 bytes. dst = NULL: only *bytes is set.
 * Errors: INVALID_ARG, BUFFER_TOO_SMALL. */
recoil_status recoil_plan_decode_table(const recoil_plan *plan, void *dst, size_t cap, size_t *bytes);
/* Launch shape used by recoil_decode for this plan (default: waves 0, i.e. 16
 * per workgroup or 1 for decodes with few runs; K = 8 groups per super-step for
 * uint8 tables, 4 for uint16; units_per_run 0). pairs_per_wave is ignored.
 * Errors: INVALID_ARG (unsupported shape). */
recoil_status recoil_plan_set_tuning(recoil_plan *plan, const recoil_tuning *tuning);
/* Autotuner for one plan: times every launch shape (waves per workgroup 1/8/16 x
 * K 4/8 x units per run 0/1/2/4) with recoil_decode on the caller's buffers,
 * `reps` timed launches each after one warm-up, keeps the fastest median and
 * leaves it set on the plan. Results are cached per process, keyed by the
 * device architecture and the stream's shape (N, M, W, symbol bytes, n).
 * Synchronises `stream`; d_out and d_error receive the last trial's decode.
 * best (may be NULL) receives the tuning (pairs_per_wave is 1); best_ms (may be
 * NULL) the winning median, or -1 when served from the cache.
 * Errors: INVALID_ARG, HIP. */
recoil_status recoil_plan_autotune(recoil_plan *plan, void *d_workspace, void *d_out, uint32_t *d_error,
                                   hipStream_t stream, uint32_t reps, recoil_tuning *best, float *best_ms);
/* The grid and runs recoil_decode would use on the current device (all zero
 * when no decode kernel runs: empty or single-symbol streams). Launches nothing.
 * Errors: INVALID_ARG, HIP (occupancy query failed). */
recoil_status recoil_plan_shape(const recoil_plan *plan, recoil_decode_shape *out);
void recoil_plan_free(recoil_plan *plan);

/*
 * Decode on the GPU (Sec. 4.1: synchronisation, decoding and cross-boundary
 * phases). Each decode unit runs on W lanes of a 64-lane wavefront (one unit
 * per wave for W = 64, two for W = 32) and writes the whole symbol groups it
 * owns (Sec. 4.1.3), so every output symbol is written by its owner. Runs of
 * consecutive units whose states are exact may also decode past their own
 * groups to the end of their last K-group super-step (the shorter run of a
 * pair up to its partner's end) and then store the same symbols into the top
 * groups of the run below: the output is the same, a few groups per run are
 * stored twice (recoil_decode_count_writes measures it).
 *
 * d_workspace: the uploaded workspace (unchanged by decoding).
 * d_out:       device buffer of N * symbol_bytes bytes, 16-byte aligned.
 * d_error:     device uint32, zeroed by the caller; RECOIL_DEVERR_* bits are
 *              OR-ed in if the data turn out to be corrupt (the kernels never
 *              read or write outside the given buffers).
 * Enqueues kernels on `stream` and returns; no allocation, no synchronisation,
 * so the call can be captured in a HIP graph.
 * Errors: INVALID_ARG, ALIGNMENT, HIP (launch failure).
 */
recoil_status recoil_decode(const recoil_plan *plan, const void *d_workspace, void *d_out,
                            uint32_t *d_error, hipStream_t stream);

/*
 * Decode an adaptive stream (recoil_encode_adaptive): as recoil_decode, with the
 * per-symbol table index d_table_index (device, N uint8, the array given to the
 * encoder). Each lane reads its symbol's index at the symbol's output offset and
 * looks the slot up in that table (one more address operation per symbol; the
 * decode arithmetic of Eq. 2 is unchanged). recoil_decode refuses adaptive
 * streams. Errors: INVALID_ARG (not adaptive, NULL index), ALIGNMENT, HIP.
 */
recoil_status recoil_decode_adaptive(const recoil_plan *plan, const void *d_workspace, const uint8_t *d_table_index,
                                     void *d_out, uint32_t *d_error, hipStream_t stream);

/*
 * Checking aid (Sec. 4.1.3 output ownership): recoil_decode with the same
 * kernels and launch shape, which also adds 1 to d_counts[i] (device uint32,
 * N entries, zeroed by the caller) for every store of symbol i; slower.
 * Errors: as recoil_decode; UNSUPPORTED for single-symbol streams (filled
 * without a decode kernel).
 */
recoil_status recoil_decode_count_writes(const recoil_plan *plan, const void *d_workspace, void *d_out,
                                         uint32_t *d_counts, uint32_t *d_error, hipStream_t stream);

/*
 * The plan's per-unit records as the decode kernels read them, 4 words per unit
 * u (0-based; unit u starts at split point u + 1, the last at the final states):
 * words available (its first read is word next - 1), first group decoded (top,
 * the anchor), highest group stored (ghi), lowest group decoded and stored (glo).
 * records = NULL: only *count (the number of units) is set.
 * cap: capacity of records in units (4 words each).
 * Errors: INVALID_ARG, BUFFER_TOO_SMALL (cap below the number of units),
 * UNSUPPORTED (records requested of a packed plan: they exist on the device only).
 */
recoil_status recoil_plan_units(const recoil_plan *plan, uint32_t *records, uint32_t cap, uint32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* RECOIL_H */
