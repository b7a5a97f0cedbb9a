/*
 * Recoil CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, deliberately unoptimised implementation of what the Recoil
 * decode path computes (Lin et al., "Recoil: Parallel rANS Decoding with
 * Decoder-Adaptive Scalability", ICPP 2023). It exists to check the product
 * library; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no code, header or table with the product path.
 *
 * Everything is parameterised (renormalisation lower bound L = 2^l_bits,
 * word size b_bits, quantisation n, lane count W) so that brute-force tests can
 * use tiny parameters. The paper's recommended set (Table "rANS parameters")
 * is l_bits = 16, b_bits = 16, n <= 16, W = 32, 32-bit states.
 *
 * Indexing is 0-based throughout (the paper counts symbols from 1).
 */
#ifndef RECOIL_ORACLE_H
#define RECOIL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t lanes;        /* W: interleaved coders, 1..64 */
    uint32_t quant_bits;   /* n: f and F sum to 2^n */
    uint32_t symbol_bytes; /* 1 or 2 */
    uint32_t alphabet;     /* symbols are 0 .. alphabet-1 */
    uint32_t l_bits;       /* L = 2^l_bits, requires n <= l_bits */
    uint32_t b_bits;       /* bits per renormalisation word, requires n <= b_bits <= 16 */
} orc_params;

typedef struct {
    uint64_t n_symbols;
    uint64_t n_words;
    uint32_t threads;       /* M: decode units; M-1 split points */
    uint32_t lanes, quant_bits, symbol_bytes, alphabet, l_bits, b_bits;
    uint64_t table_bytes, metadata_bytes, total_bytes;
} orc_info;

/* One renormalisation event: the encoder emitted word `pos` for lane `lane`,
 * after encoding that lane's symbol `idx`; `state` is the post-shift state. */
typedef struct {
    uint64_t pos;
    uint32_t lane;
    int64_t idx;
    uint32_t state;
} orc_event;

enum {
    ORC_OK = 0,
    ORC_BAD_PARAM = -1,
    ORC_INFEASIBLE = -2,
    ORC_CORRUPT = -3,
    ORC_SMALL_BUFFER = -4,
};

/* Frequency quantisation (see oracle.cpp for the rule). */
int orc_quantize(const uint64_t *counts, uint32_t alphabet, uint32_t n, uint32_t *f_out);

/* Encode and pick M-1 split points; the encoder handle keeps everything. */
typedef struct orc_enc orc_enc;
int orc_encode(const void *symbols, uint64_t n_symbols, const orc_params *p,
               const uint32_t *freq /* NULL: quantise from the data */,
               uint32_t threads, orc_enc **out);
/* Adaptive coding (Sec. 3.1): `tables` frequency tables (freqs: tables x alphabet,
 * each summing to 2^n) and symbol i coded with table tidx[i] (< tables). The
 * container (magic "RCA1") carries the tables; the index array is side information
 * that decoding needs again (orc_set_table_index). */
int orc_encode_adaptive(const void *symbols, uint64_t n_symbols, const orc_params *p,
                        const uint32_t *freqs, uint32_t tables, const uint8_t *tidx,
                        uint32_t threads, orc_enc **out);
void orc_enc_free(orc_enc *e);
uint64_t orc_enc_container_size(const orc_enc *e);
int orc_enc_container(const orc_enc *e, uint8_t *dst, uint64_t cap);
uint32_t orc_enc_threads(const orc_enc *e);
uint64_t orc_enc_num_events(const orc_enc *e);
int orc_enc_events(const orc_enc *e, orc_event *dst, uint64_t cap);
uint64_t orc_enc_num_candidates(const orc_enc *e);
/* Split point k (1 .. M-1): word position, Imax, Imin, W states, W symbol indices. */
int orc_enc_split(const orc_enc *e, uint32_t k, uint64_t *pos, int64_t *imax, int64_t *imin,
                  uint32_t *states, int64_t *indices);
/* The candidate that word `pos` would give (valid=0 if some lane has no event yet). */
int orc_enc_candidate_at(const orc_enc *e, uint64_t pos, int *valid, int64_t *imax,
                         int64_t *imin, uint32_t *states, int64_t *indices);

/* Backward scan on a synthetic event log: the split at event `split_event`
 * records, for each lane, its latest event at or before that word. */
int orc_scan_events(const orc_event *events, uint64_t n_events, uint32_t lanes,
                    uint64_t split_event, uint32_t *states, int64_t *indices, int *valid);

/* Bit-packed data series (MSB first). `width_field` is the size of the
 * leading (width-1) field; signed series carry one sign bit per value. */
int orc_series_pack(const int64_t *values, uint64_t count, uint32_t width_field, int is_signed,
                    uint8_t *dst, uint64_t cap_bytes, uint64_t *n_bits);
int orc_series_unpack(const uint8_t *src, uint64_t n_bytes, uint64_t count,
                      uint32_t width_field, int is_signed, int64_t *values, uint64_t *n_bits);

/* Assemble a container from explicit parts (used to check the metadata
 * layout against the paper's worked example). split_states / split_indices
 * hold (threads-1) rows of `lanes` values. */
int orc_assemble(const orc_params *p, uint64_t n_symbols, const uint32_t *freq,
                 const uint16_t *words, uint64_t n_words, const uint32_t *final_states,
                 uint32_t threads, const uint64_t *split_pos, const uint32_t *split_states,
                 const int64_t *split_indices, uint8_t *dst, uint64_t cap, uint64_t *written);

/* Conventional partitioning (Sec. 2.3), the comparison baseline: `partitions`
 * contiguous sub-sequences of S = ceil(N / partitions) symbols rounded up to whole
 * groups of W (fewer sub-sequences if that covers N), each coded independently
 * from state L with the one table, sub-bitstreams concatenated. Container magic
 * "RCP1" (see oracle.cpp). dst = NULL: only *written (the size) is set.
 * Threads of the decoders below are the sub-sequences; combining is refused. */
int orc_encode_partitioned(const void *symbols, uint64_t n_symbols, const orc_params *p,
                           const uint32_t *freq, uint32_t partitions, uint8_t *dst, uint64_t cap,
                           uint64_t *written);

/* Container-level operations. */
int orc_info_of(const uint8_t *c, uint64_t len, orc_info *out);
int orc_combine(const uint8_t *c, uint64_t len, uint32_t target_threads, uint8_t *dst,
                uint64_t cap, uint64_t *written);

typedef struct orc_dec orc_dec;
int orc_open(const uint8_t *c, uint64_t len, orc_dec **out);
void orc_close(orc_dec *d);
/* Adaptive containers only: the per-symbol table index (n = N entries, each < tables). */
int orc_set_table_index(orc_dec *d, const uint8_t *tidx, uint64_t n);
/* Serial interleaved decode of the whole stream; checks end states and cursor. */
int orc_decode_serial(const orc_dec *d, void *out);
/* Thread t (1..M) writes only its own output range of the N-symbol buffer.
 * aligned=0: [Imin_{t-1}, Imin_t - 1]; aligned=1: whole symbol groups. */
int orc_decode_thread(const orc_dec *d, uint32_t t, int aligned, void *out);
/* Same, also listing every symbol index the thread decodes, in order,
 * including the synchronisation-phase symbols that are thrown away. */
int orc_decode_thread_trace(const orc_dec *d, uint32_t t, int aligned, void *out,
                            int64_t *decoded, uint64_t cap, uint64_t *count);
/* Output range of thread t (inclusive lo, exclusive hi). */
int orc_thread_range(const orc_dec *d, uint32_t t, int aligned, uint64_t *lo, uint64_t *hi);
/* All threads, distributed over `workers` std::threads (>= 1). */
int orc_decode_all(const orc_dec *d, int aligned, uint32_t workers, void *out);

#ifdef __cplusplus
}
#endif

#endif
