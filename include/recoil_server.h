/*
 * librecoil serving loop: the content-delivery use case of Recoil (Lin et al.,
 * ICPP 2023, Sec. 3.3 and Sec. 6). Content is encoded once at the largest
 * parallelism and kept resident in device memory; each request names a content
 * and the number of decode units the client can use. The server shrinks the
 * split metadata to that count (the combine of Sec. 3.3), admits the request when
 * its output and metadata fit the device budget, and folds every admitted
 * request that is ready into one persistent batched launch (continuous batching
 * across up to `hip_streams` launches in flight). Completion is observed through
 * a HIP event per launch.
 *
 * Work items: a request is cut into items of tuning.waves x pairs_per_wave unit
 * pairs, or smaller ones (about one per resident workgroup) when the launch's
 * pairs would not fill the resident workgroups, so that a lightly loaded launch
 * spreads each request over many CUs. A W = 32 request of at most tuning.waves
 * units decodes one unit per wave.
 *
 * Memory: the caller owns one device arena. Its first `resident_bytes` hold the
 * content (bitstream words and decode tables, copied by
 * recoil_server_add_content); the server keeps a small control region per launch
 * slot after it; everything else is the request budget (outputs plus per-request
 * unit records). A request's output stays allocated until recoil_server_release.
 *
 * Threads: one launcher thread owns the streams, events and the budget; a pool of
 * `prep_threads` host threads combines and plans requests as they arrive. All
 * entry points are thread-safe. The launcher polls its events while launches are
 * in flight, so it keeps one host core busy under load.
 *
 * Requests are admitted in submission order within two classes. A "long" request
 * (few decode units for its size: more than long_unit_bytes of output per unit)
 * decodes serially for a long time, and a launch keeps its stream until its
 * slowest request ends, so launches holding long requests may occupy at most
 * long_streams of the streams; short requests pass waiting long ones. A request
 * that does not fit the budget waits (and holds back later ones) until outputs
 * are released or launches finish; one that cannot fit even in an empty budget
 * completes with RECOIL_ERR_BUFFER_TOO_SMALL.
 */
#ifndef RECOIL_SERVER_H
#define RECOIL_SERVER_H

#include "recoil.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct recoil_server recoil_server;

typedef struct {
    uint32_t hip_streams;       /* launches in flight at once, 1..8 (each on its own default-priority stream) */
    uint32_t max_batch;         /* most requests folded into one launch, 1..4096 */
    uint32_t prep_threads;      /* host threads that combine and plan requests, 1..64 */
    uint32_t items_per_launch;  /* work-item capacity of one launch, 1024..2^22 */
    uint64_t resident_bytes;    /* arena bytes at its start reserved for content */
    recoil_tuning tuning;       /* launch shape of the batched kernel (recoil_default_tuning()) */
    uint64_t long_unit_bytes;   /* a request with more output bytes per decode unit is "long" (0: 131072) */
    uint32_t long_streams;      /* most launches holding long requests in flight (0: hip_streams / 2, >= 1) */
    uint32_t reserved;
} recoil_server_config;

typedef struct {
    uint64_t request_id;
    uint64_t tag;               /* the caller's value from recoil_server_submit */
    uint32_t content;
    uint32_t splits;            /* decode units after combining */
    int32_t status;             /* RECOIL_OK, or why the request was not decoded */
    uint32_t device_error;      /* RECOIL_DEVERR_* bits raised by its launch (0 when clean) */
    uint64_t out_offset;        /* bytes from the arena base to the decoded symbols (256-byte aligned) */
    uint64_t out_bytes;         /* n_symbols * symbol_bytes */
    uint64_t metadata_bytes;    /* packed split metadata after combining (what a client would receive) */
    uint64_t t_arrival_ns;      /* recoil_server_now_ns() clock */
    uint64_t t_admit_ns;        /* budget granted */
    uint64_t t_launch_ns;       /* its launch was enqueued */
    uint64_t t_done_ns;         /* the launcher saw its launch's completion event */
} recoil_completion;

typedef struct {
    uint64_t submitted, completed, rejected, launches, requests_launched;
    uint64_t pending;           /* submitted, not yet launched */
    uint64_t in_flight;         /* launches enqueued, not yet complete */
    uint64_t budget_bytes, budget_used, budget_peak;
    uint64_t resident_used;
    uint64_t decoded_bytes;     /* output bytes of completed requests */
} recoil_server_stats;

/* Monotonic clock (nanoseconds) used for every timestamp of the server. */
uint64_t recoil_server_now_ns(void);

/*
 * Create a server over the caller's arena (256-byte aligned; it must stay valid
 * until recoil_server_destroy returns) on the current HIP device.
 * Errors: INVALID_ARG (bad config, arena too small for the control regions),
 * ALIGNMENT, HIP.
 */
recoil_status recoil_server_create(const recoil_server_config *cfg, void *d_arena, size_t arena_bytes,
                                   recoil_server **out);

/*
 * Make a blob servable: copies its words and decode table into the resident
 * region (synchronously) and keeps a reference to its split metadata. The blob
 * may be freed afterwards. Errors: INVALID_ARG, UNSUPPORTED (W not 32/64, n outside 8..16,
 * or a partitioned blob, whose units cannot be combined per request, or an adaptive
 * blob, which is decoded alone; 13 <= n <= 16 content is served, its requests' items
 * by a second persistent launch per admitted set), BUFFER_TOO_SMALL
 * (resident region full), HIP.
 */
recoil_status recoil_server_add_content(recoil_server *server, const recoil_blob *blob, uint32_t *content_id);

/*
 * Queue a request for `content` decoded with at most `splits` units (0 or more
 * than the content holds: all of them). arrival_ns: the request's arrival time on
 * the recoil_server_now_ns clock (0: now); latency is measured from it.
 * Errors: INVALID_ARG (unknown content, or the server is shutting down).
 */
recoil_status recoil_server_submit(recoil_server *server, uint32_t content, uint32_t splits, uint64_t tag,
                                   uint64_t arrival_ns, uint64_t *request_id);

/*
 * Copy up to `cap` completions (oldest first) into `done`, waiting up to
 * timeout_us microseconds for the first one. Returns the number copied.
 */
uint32_t recoil_server_poll(recoil_server *server, recoil_completion *done, uint32_t cap, uint32_t timeout_us);

/* Return a completed request's output to the budget. Errors: INVALID_ARG (unknown or already released). */
recoil_status recoil_server_release(recoil_server *server, uint64_t request_id);

recoil_status recoil_server_get_stats(const recoil_server *server, recoil_server_stats *stats);

/*
 * Stop accepting requests, drop those not yet launched, wait for launches in
 * flight, join the threads and free host resources (the arena stays the caller's).
 */
void recoil_server_destroy(recoil_server *server);

#ifdef __cplusplus
}
#endif

#endif /* RECOIL_SERVER_H */
