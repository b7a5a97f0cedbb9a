/*
 * librecoil batched decoding: many independent Recoil streams decoded by one
 * persistent launch, the one-launch-per-stream baseline, HIP graph capture and
 * the autotuner. Same conventions as recoil.h (library-owned host objects,
 * caller-owned device memory, recoil_status results).
 *
 * This is an extension of the paper's single-stream decoder (Lin et al., ICPP
 * 2023, Sec. 4.1): the per-unit arithmetic is unchanged; only scheduling across
 * streams is added.
 */
#ifndef RECOIL_BATCH_H
#define RECOIL_BATCH_H

#include "recoil.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct recoil_batch recoil_batch;
typedef struct recoil_graph recoil_graph;

recoil_tuning recoil_default_tuning(void);

/*
 * Plan a batch of `count` blobs (each W = 32 or 64, 8 <= n <= 12). Reports the device
 * workspace size (words, tables, unit records, stream descriptors, work items,
 * queue counter) and the output size: stream i's symbols land at the offset given
 * by recoil_batch_output_offset (256-byte aligned). tuning: NULL for the default.
 * Streams with 13 <= n <= 16 (two-level tables) form a table class decoded by a
 * launch of its own. Errors: INVALID_ARG, UNSUPPORTED (see recoil_plan_create; also
 * adaptive streams, which are decoded alone).
 */
recoil_status recoil_batch_create(const recoil_blob *const *blobs, uint32_t count, const recoil_tuning *tuning,
                                  recoil_batch **out, size_t *workspace_bytes, size_t *output_bytes);
void recoil_batch_free(recoil_batch *batch);
recoil_status recoil_batch_output_offset(const recoil_batch *batch, uint32_t index, uint64_t *offset, uint64_t *bytes);
uint32_t recoil_batch_items(const recoil_batch *batch);

/* Asynchronous H2D copy of everything into d_workspace (256-byte aligned).
 * Errors: INVALID_ARG, BUFFER_TOO_SMALL, ALIGNMENT, HIP. */
recoil_status recoil_batch_upload(const recoil_batch *batch, void *d_workspace, size_t bytes, hipStream_t stream);

/* Change the launch shape; rebuilds the work items on the host and, if
 * d_workspace is not NULL, re-uploads them on `stream`. Errors: INVALID_ARG, HIP. */
recoil_status recoil_batch_set_tuning(recoil_batch *batch, const recoil_tuning *tuning, void *d_workspace,
                                      hipStream_t stream);
recoil_status recoil_batch_get_tuning(const recoil_batch *batch, recoil_tuning *tuning);

/* One persistent launch per decode-table class that has streams (tables up to
 * 16 KiB, i.e. uint8 with n <= 12; larger tables), each with LDS for its own
 * class's largest table, in that order; a one-thread kernel resets the class's
 * queue counter in the workspace before each. d_out: output base (>= output_bytes);
 * d_error: zeroed device word (RECOIL_DEVERR_* bits). Enqueue-only, capturable.
 * Errors: INVALID_ARG, HIP. */
recoil_status recoil_decode_batch(const recoil_batch *batch, void *d_workspace, void *d_out, uint32_t *d_error,
                                  hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): recoil_decode_batch with
 * the queue heads in a statically allocated device array of the library instead
 * of the workspace, so d_workspace is only read. The array is 384 bytes per GPU
 * (one head for each of the three table classes, 128 bytes apart), held by every GPU the library runs
 * on until the process ends; each launch's head is reset by a kernel, not a
 * memset. The first call on a device looks up the array's address on that device
 * (hipGetSymbolAddress, current device), so make it outside graph capture. Calls
 * that overlap on one GPU share the heads and race: serialise them (one stream, or
 * events). Allocates nothing, synchronises nothing. Arguments and output as
 * recoil_decode_batch. Errors: INVALID_ARG, UNSUPPORTED (more table classes than
 * heads; not produced by recoil_batch_create), HIP.
 */
recoil_status recoil_decode_batch_noalloc(const recoil_batch *batch, const void *d_workspace, void *d_out,
                                          uint32_t *d_error, hipStream_t stream);

/* Baseline: the single-stream decoder launched once per stream, in order, on `stream`. */
recoil_status recoil_decode_batch_per_stream(const recoil_batch *batch, const void *d_workspace, void *d_out,
                                             uint32_t *d_error, hipStream_t stream);

/* Capture the [queue reset; persistent decode] pair of every class for these buffers in a HIP graph
 * (captured on a private stream) and instantiate it. Replay with recoil_graph_launch.
 * Errors: INVALID_ARG, HIP. */
recoil_status recoil_batch_graph_create(const recoil_batch *batch, void *d_workspace, void *d_out, uint32_t *d_error,
                                        recoil_graph **out);
recoil_status recoil_graph_launch(recoil_graph *graph, hipStream_t stream);
void recoil_graph_free(recoil_graph *graph);

/*
 * Autotuner: times every launch shape (waves 8/16 x K 4/8 x pairs per wave
 * 1/2/4/8 x units per run 1/2/4/8, shapes that do not fit the CU skipped) on this batch, `reps` timed
 * launches each after one warm-up, keeps the fastest median and leaves it set on
 * the batch (work items re-uploaded). Results are cached per process, keyed by the
 * device architecture and the batch's shape. Synchronises `stream`.
 * best_ms receives the winning median (-1 when served from the cache).
 * Errors: INVALID_ARG, HIP.
 */
recoil_status recoil_autotune(recoil_batch *batch, void *d_workspace, void *d_out, uint32_t *d_error,
                              hipStream_t stream, uint32_t reps, recoil_tuning *best, float *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* RECOIL_BATCH_H */
