/*
 * hc.h -- exact clustering of Timepix pixel hits on one AMD MI355X (gfx950).
 *
 * Method: Celko, Mraz, Bergmann, Manek, "Parallel CPU- and GPU-based connected
 * component algorithms for event building for hybrid pixel detectors"
 * (arXiv 2412.11809).
 *
 *   Hit record .............. Section 1: pixel coordinates x, y; time of
 *                             arrival (ToA); time over threshold (ToT).
 *   Cluster ................. Section 2, conditions (i), (ii), (iii)(a): a
 *                             maximal set of hits joined by a path whose every
 *                             step is between 8-neighbouring (or identical)
 *                             pixels and whose ToAs differ by at most dt.
 *   Parallel method ......... Section 4.1 and its Algorithm "High-level GPU
 *                             clustering": sort by ToA, search a hit's own
 *                             pixel and its eight neighbours for the latest
 *                             earlier hit, and join clusters with a
 *                             union-find forest with path compression.
 *   Features ................ Sections 1 and 6 motivate per-cluster features;
 *                             the set below is this library's.
 *
 * Conventions shared by every entry point
 *   - Device pointers are HIP device memory (e.g. torch CUDA tensors on ROCm);
 *     the caller owns every buffer, the library never frees caller memory.
 *   - dt is in ToA ticks and inclusive (|toa_a - toa_b| <= dt); dt =
 *     UINT64_MAX means "no time limit".  Saturating arithmetic throughout.
 *   - labels[i] is the smallest input index of hit i's cluster (unique and
 *     independent of scheduling).  features[k] is the k-th cluster in
 *     ascending label order; the features buffer must hold n records.
 *   - Calls are asynchronous on opts->stream (NULL = the null stream).
 *     Argument errors return a negative HC_ERR_* synchronously.  Errors found
 *     in the data (a hit outside the sensor) are reported asynchronously:
 *     *n_clusters (device memory) then holds HC_ERR_RANGE.
 *   - Calls on distinct workspaces/streams are independent; two calls that
 *     share a workspace must be ordered by the caller (same stream).  With a
 *     NULL workspace the library keeps one cached buffer per (device,
 *     stream): calls on different streams never share it, and calls on one
 *     stream are ordered by that stream, from any number of host threads.
 */
#ifndef HC_H
#define HC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One pixel hit (Section 1), 16 bytes: ToA in detector ticks, pixel column x,
 * row y, ToT, and a reserved field that is ignored. */
typedef struct {
    uint64_t toa;
    uint16_t x, y, tot, reserved;
} hc_hit;

/* Features of one cluster, 64 bytes.  All integer fields are exact sums,
 * minima or maxima over the cluster's hits.  cx = (double)sum_x_tot /
 * (double)sum_tot (likewise cy), correctly rounded; if every ToT of the
 * cluster is zero the centroid is the unweighted mean of x (y). */
typedef struct {
    int32_t label;      /* smallest input index in the cluster */
    uint32_t size;      /* number of hits */
    uint64_t sum_tot;   /* sum of ToT */
    uint64_t toa_min;   /* earliest ToA */
    uint64_t toa_max;   /* latest ToA */
    uint64_t sum_x_tot; /* sum of x * ToT */
    uint64_t sum_y_tot; /* sum of y * ToT */
    double cx, cy;      /* ToT-weighted centroid in pixel units */
} hc_features;

/* Options; pass NULL for the defaults (256 x 256 sensor, disorder hint 4096,
 * internal workspace, null stream). */
typedef struct {
    uint32_t width, height;  /* sensor size in pixels, each 1..65535 */
    uint32_t disorder_hint;  /* expected max positional displacement of a hit
                                from its ToA-sorted place (the paper's
                                partial orderliness, Section 3.1).  A tuning
                                hint only: wrong values cost speed, never
                                exactness. 0 = 4096. */
    uint32_t flags;          /* 0, or one HC_FLAG_LINK_* value; hc_cluster also
                                takes HC_FLAG_GLOBAL_TIME */
    void* workspace;         /* device scratch of >= hc_workspace_size bytes,
                                or NULL: the library then keeps a cached
                                buffer per (device, stream), grown with
                                hipMalloc and kept until the process ends */
    size_t workspace_bytes;
    void* stream;            /* hipStream_t to run on; NULL = null stream */
} hc_opts;

/* Neighbour search variant (results are identical).  By default every tile
 * goes through a pixel index (occupancy bitmap + per-pixel lists in LDS) when
 * the sensor has at most 448 x 512 pixels, and scans each hit's dt window
 * backwards on larger sensors (up to 16384 x 16384; beyond both, tiles take
 * a slower path).  The flags force one of the two for every tile. */
#define HC_FLAG_LINK_PIXEL_INDEX 1u
#define HC_FLAG_LINK_WINDOW 2u

/* hc_cluster only: cluster by the paper's second definition, Section 2
 * (iii)(b), the dynamic global-time neighbourhood: a cluster is a maximal
 * (under inclusion) set of hits that is spatially connected through
 * 8-neighbouring or identical pixels at any ToA, and whose ToAs, in order,
 * leave no gap larger than dt (every hit but the earliest has another hit of
 * the cluster at most dt before it).  Every cluster of the default definition
 * (iii)(a) lies inside one of these.  Labels and features keep their
 * conventions.  The device refines a partition in rounds until it no longer
 * changes; the call waits for the stream after every round, so it returns
 * once the work is done (hc_workspace_size grows accordingly). */
#define HC_FLAG_GLOBAL_TIME 4u

enum {
    HC_OK = 0,
    HC_ERR_ARG = -1,       /* bad argument (NULL pointer, n < 0, bad size) */
    HC_ERR_RANGE = -2,     /* a hit has x >= width or y >= height */
    HC_ERR_WORKSPACE = -3, /* workspace smaller than hc_workspace_size */
    HC_ERR_DEVICE = -4,    /* HIP runtime error (see hc_last_error) */
    HC_ERR_DISORDER = -5,  /* stream: a hit violates the disorder contract */
    HC_ERR_OVERFLOW = -6,  /* more than 2^31 - 1 hits in one labelling */
    HC_ERR_BUDGET = -7,    /* server: request exceeds the memory budget */
    HC_ERR_BUSY = -8       /* server: shutting down, or still busy at a wait's timeout */
};

/* Bytes of device workspace hc_cluster needs for n hits with these options. */
size_t hc_workspace_size(const hc_opts* opts, int64_t n);

/* Cluster n hits (device array, any order) with time window dt.
 * Writes labels[n] (device), features[0..K) (device, capacity n) and
 * *n_clusters = K (device int32; or HC_ERR_RANGE, see above).
 * features may be NULL to skip the feature table (K is still written).
 * Returns HC_OK once all work is enqueued, or a negative HC_ERR_* for an
 * argument/runtime error (nothing is then guaranteed about the outputs). */
int hc_cluster(const hc_hit* hits, int32_t n, uint64_t dt, int32_t* labels,
               hc_features* features, int32_t* n_clusters, const hc_opts* opts);

/* hc_cluster without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as hc_cluster; the
 * workspace is a fixed scratch array of HC_NOALLOC_SCRATCH_BYTES in device
 * memory, which each GPU the library runs on holds until the process ends.
 * opts->workspace must be NULL and HC_FLAG_GLOBAL_TIME is rejected
 * (HC_ERR_ARG).  A call whose workspace (hc_workspace_size for the same n and
 * options) exceeds the array returns HC_ERR_WORKSPACE, before any device
 * work: about 1.3 million hits fit.  Every call on one GPU shares that GPU's
 * array, whatever stream it runs on, so calls that overlap in time on one GPU
 * race and return wrong results: the caller serialises them (one stream, or
 * an event between them).  The first call on a device looks the array's
 * address up; later calls allocate nothing, neither device nor pinned host
 * memory. */
#define HC_NOALLOC_SCRATCH_BYTES (256ull << 20)
int hc_cluster_noalloc(const hc_hit* hits, int32_t n, uint64_t dt, int32_t* labels,
                       hc_features* features, int32_t* n_clusters, const hc_opts* opts);
/* Size of that scratch array in bytes (HC_NOALLOC_SCRATCH_BYTES). */
size_t hc_noalloc_scratch_bytes(void);

/* ---- Per-cluster products ------------------------------------------------
 *
 * Computed on the device from what hc_cluster wrote (labels, feature table,
 * cluster count), for the steps the paper places around the clustering:
 *   - the bounding box of every cluster: the smallest sensor-aligned
 *     rectangle holding its hits (Section 3.3, second test of the merge
 *     cascade);
 *   - a filter that keeps the clusters whose size, ToT sum and first ToA lie
 *     in closed ranges (Section 3.1, cluster outputting: filtering to reduce
 *     the data volume; Section 6: filtering on the GPU);
 *   - the hits of the kept clusters grouped cluster by cluster, one block of
 *     memory per cluster (step 6 of the paper's high-level GPU algorithm);
 *     blocks follow the kept rows, hits inside a block keep their input
 *     order. */
typedef struct {
    uint16_t x_min, x_max, y_min, y_max; /* inclusive pixel ranges */
} hc_box;

typedef struct {
    uint32_t min_size, max_size;       /* min_size <= size <= max_size */
    uint64_t min_sum_tot, max_sum_tot; /* min_sum_tot <= sum_tot <= max_sum_tot */
    uint64_t toa_from, toa_to;         /* toa_from <= toa_min <= toa_to */
} hc_filter;

/* Bytes of device workspace hc_cluster_products needs for n hits. */
size_t hc_products_workspace_size(int64_t n);

/* hits[n], labels[n], features[0..K) and *n_clusters = K: device buffers as
 * hc_cluster wrote them (same hits).  filter: NULL keeps every cluster.
 * Outputs (device):
 *   boxes[K]       box of every feature row, or NULL to skip;
 *   keep_rows[K]   the kept feature rows, ascending; *n_keep = their number
 *                  (or HC_ERR_DEVICE if the inputs are inconsistent);
 *   grouped[n], grouped_idx[n]  the kept clusters' hits (and their input
 *                  indices), block by block; either may be NULL (both NULL
 *                  skips the grouping);
 *   row_start[K+1] start of every kept block in grouped, then the total
 *                  (entries 0..n_keep), or NULL.
 * workspace: device memory of >= hc_products_workspace_size(n) bytes.
 * Asynchronous on `stream` (a hipStream_t, NULL = the null stream). */
int hc_cluster_products(const hc_hit* hits, int32_t n, const int32_t* labels, const hc_features* features,
                        const int32_t* n_clusters, const hc_filter* filter, hc_box* boxes,
                        int32_t* keep_rows, int32_t* n_keep, hc_hit* grouped, int32_t* grouped_idx,
                        int64_t* row_start, void* workspace, size_t workspace_bytes, void* stream);

/* ---- Stream form: one detector's hit stream, pushed chunk by chunk --------
 *
 * The stream is "t-ordered" (paper, Section 3.1): for any two hits i < j in
 * push order, toa_i < toa_j + t, with t = max_disorder_ticks.  Clusters that
 * straddle chunk borders (the paper's border and open clusters, Section 3.3;
 * border grouping, step 5 of its high-level GPU algorithm) are stitched
 * exactly: open hits stay on the device and are clustered again with the
 * next chunk.  With M the largest ToA pushed so far, every later hit has
 * toa > M - t; a cluster is closed -- its labels final, its features emitted
 * (Algorithm "processHit", closeAndDispatchOldClusters) -- once
 * toa_max + dt <= M - t.  While M < t there is no such bound yet: nothing
 * is rejected for its ToA and nothing closes before the flush.
 *
 * Labels are stream-global: the smallest global index (0-based position in
 * the concatenation of all accepted chunks) of the hit's cluster.  They are
 * written into each chunk's labels buffer as its clusters close, possibly
 * during a later push or the flush; a chunk is complete when its tag is
 * reported by hc_stream_poll.  At most 2^31 - 1 hits per stream.
 *
 * Pushes are asynchronous: the stream's state (open hits, M, the next global
 * index) lives on the device, each chunk is accepted or rejected there, and
 * hc_stream_push returns once the push is enqueued (it waits only while
 * several pushes are already in flight, or when buffers must grow).  Results
 * arrive through hc_stream_poll.  A stream is single-producer; all its work
 * runs on opts->stream, so work the caller enqueues later on that stream is
 * ordered after every push. */
typedef struct hc_stream hc_stream;

/* opts: sensor size, disorder_hint (positional, for the sort), stream; the
 * workspace fields are ignored (the stream owns its device buffers). */
int hc_stream_create(const hc_opts* opts, uint64_t dt, uint64_t max_disorder_ticks, hc_stream** out);

/* Append n hits (device array, read when the push runs on the stream: keep
 * it unchanged until then -- later work on the same stream is ordered after
 * it, and hc_stream_wait waits for it).  labels: device int32[n] that the
 * library fills as the chunk's clusters close; it must stay valid until
 * `tag` is returned by hc_stream_poll.  The chunk is rejected on the device,
 * leaving the stream unchanged and its labels untouched, if a hit is off the
 * sensor (status HC_ERR_RANGE) or has toa <= M - t (when M >= t) or, after a
 * flush, toa <= F (see hc_stream_flush) (status HC_ERR_DISORDER); the status
 * comes with the tag from hc_stream_poll.  Returns HC_OK once enqueued,
 * HC_ERR_ARG for bad arguments, HC_ERR_OVERFLOW past 2^31 - 1 hits pushed,
 * HC_ERR_DEVICE after a device failure. */
int hc_stream_push(hc_stream* s, const hc_hit* hits, int32_t n, int32_t* labels, uint64_t tag);

/* Several chunks in one push: k (1..16) chunks stored back to back at hits
 * (device memory), chunk j with counts[j] > 0 hits, its labels to labels[j]
 * (device int32[counts[j]]) and reported under tags[j]; counts, labels and
 * tags are host arrays, read before the call returns.  The result is that of
 * k hc_stream_push calls in order -- each chunk accepted or rejected on its
 * own, against the watermark the chunks before it set -- with one pass of
 * device work, which spares small chunks the fixed cost of a push (the
 * serving loop merges queued chunks of a stream this way).  Not for streams
 * that take ids (HC_ERR_ARG). */
int hc_stream_push_chunks(hc_stream* s, const hc_hit* hits, int32_t k, const int32_t* counts,
                          int32_t* const* labels, const uint64_t* tags);

/* hc_stream_push with caller-chosen ids (device int32[n], non-negative):
 * a cluster's label -- in the labels buffers and in the closed features --
 * is then the smallest id among its hits instead of the smallest global
 * index.  For callers that push hits in another order than they number them
 * (the buffer filling of hc_ingest moves late hits into the next buffer).  A
 * stream takes ids with every push or with none (HC_ERR_ARG otherwise); a
 * chunk with a negative id is rejected (status HC_ERR_ARG). */
int hc_stream_push_ids(hc_stream* s, const hc_hit* hits, const int32_t* ids, int32_t n, int32_t* labels,
                       uint64_t tag);

/* Drain completion events into HOST buffers, without waiting for pushes in
 * flight: up to cap tags of finished chunks (in completion order) with their
 * status (status may be NULL): HC_OK when every label of the chunk is final,
 * or the reason it was rejected; and up to closed_cap features of closed
 * clusters (labels stream-global; ascending label within one push).
 * Entries beyond the caps stay queued for the next call. */
int hc_stream_poll(hc_stream* s, uint64_t* done_tags, int32_t* status, int32_t cap, int32_t* n_done,
                   hc_features* closed, int32_t closed_cap, int32_t* n_closed);

/* Wait until every push enqueued so far has run on the device (their
 * completions are then available to hc_stream_poll). */
int hc_stream_wait(hc_stream* s);

/* Pre-allocate the stream's device buffers for chunks of up to max_chunk
 * hits (plus a margin of open hits), so that later pushes allocate nothing
 * unless a chunk is larger or unusually many clusters stay open. */
int hc_stream_reserve(hc_stream* s, int32_t max_chunk);

/* Hits held open on the device (their clusters may still grow) after the
 * last push known to have completed; -1 for a NULL stream. */
int64_t hc_stream_open_hits(const hc_stream* s);

/* Close every open cluster (end of stream) and wait for it; afterwards all
 * pushed chunks are complete.  The stream may continue as a new segment that
 * no cluster spans:
 * with M the largest ToA pushed before the flush, a later push is rejected
 * (HC_ERR_DISORDER) unless every hit has toa > F = M + dt (saturating), so no
 * later hit can be adjacent in time to a hit whose label is already final. */
int hc_stream_flush(hc_stream* s);

void hc_stream_destroy(hc_stream* s);

/* ---- Host ingest front end ------------------------------------------------
 *
 * Hits as the detector delivers them (host memory, t-ordered, Section 3.1),
 * numbered by arrival (0, 1, 2, ... over all feeds), are filled into pinned
 * buffers by the paper's buffer filling (its Algorithm "Hit buffer filling",
 * Section 4.1): a buffer takes every hit until it holds b - b_t, tracking the
 * largest ToA seen (toa_max); after that only hits with
 * toa < toa_max + t_closing, later ones going to the next buffer; when a hit
 * arrives with toa - toa_max > t + t_closing the buffer is complete and is
 * sent (so is a buffer whose next buffer is full).  Sent buffers are copied
 * to the device on their own HIP stream and clustered by an hc_stream
 * (exact stitching across buffers) while the next ones fill and copy
 * (steps 1, 2 and 8 of the paper's high-level GPU algorithm; pinned memory
 * and copy/compute overlap, Section 5).  labels_out[i] receives the smallest
 * arrival index of hit i's cluster once final; hc_ingest_finish makes every
 * fed hit final. */
typedef struct hc_ingest hc_ingest;

typedef struct {
    uint32_t width, height;      /* sensor (0 => 256) */
    uint32_t disorder_hint;      /* positional displacement hint (0 => 4096) */
    uint32_t flags;              /* must be 0 */
    uint64_t dt;                 /* time window of the clusters, ticks */
    uint64_t max_disorder_ticks; /* t of the input (t-ordered bound) */
    uint64_t t_closing;          /* the paper's t_closing: longest expected cluster duration */
    int32_t buffer_hits;         /* b: capacity of one buffer */
    int32_t reserve_hits;        /* b_t: hits expected within t + t_closing (0 <= b_t < b) */
    int32_t n_buffers;           /* pinned/device buffer pairs (0 => 4; at least 3) */
    int32_t reserved;            /* must be 0 */
    void* stream;                /* hipStream_t of the clustering (NULL = null stream) */
} hc_ingest_config;

typedef struct {
    int64_t hits_fed, hits_done;  /* numbered so far; with their labels placed */
    int64_t buffers_sent, buffers_done;
    int64_t forced_sends;         /* buffers sent because the next one was full */
    int64_t diverted;             /* hits that arrived for the next buffer before this one was sent */
    int64_t waits;                /* times the host waited for a free buffer */
} hc_ingest_stats;

/* labels_out: HOST int32[labels_cap]; feeding more hits returns HC_ERR_OVERFLOW. */
int hc_ingest_create(const hc_ingest_config* cfg, int32_t* labels_out, int64_t labels_cap, hc_ingest** out);
/* Number and buffer n more hits (host array, arrival order); sends buffers as
 * they complete and places the labels of finished ones.  Never waits for the
 * device unless every buffer is in use. */
int hc_ingest_feed(hc_ingest* g, const hc_hit* hits, int64_t n);
/* Send what is buffered, close every cluster and wait: afterwards every fed
 * hit has its final label.  Later feeds start a new segment (see
 * hc_stream_flush). */
int hc_ingest_finish(hc_ingest* g);
int hc_ingest_stats_read(const hc_ingest* g, hc_ingest_stats* out);
void hc_ingest_destroy(hc_ingest* g);

/* ---- Batch form: many independent chunks, one launch per stage ----------
 *
 * Chunks of uneven size (e.g. from several detectors) are clustered
 * independently, each with its own dt, by ONE sequence of launches whose
 * tiles cover all chunks (tiles never straddle two chunks), so small and large
 * chunks load the GPU evenly.  The paper partitions hits into chunks, one per
 * thread (step 4 of its high-level GPU algorithm); here chunks are independent
 * inputs and every chunk is cut into tiles.
 *
 * hits:       device array, the chunks one after another
 * offsets:    HOST int64[n_chunks + 1], chunk c = hits[offsets[c], offsets[c+1])
 * dts:        HOST uint64[n_chunks], time window of every chunk (ticks)
 * labels:     device int32[n]: chunk-local labels (smallest index within the
 *             chunk of the hit's cluster)
 * features:   device hc_features[n] or NULL: chunk c's clusters at rows
 *             offsets[c] .. offsets[c] + n_clusters[c] - 1, ascending label
 * n_clusters: device int32[n_chunks] (or an error status per chunk)
 * plan:       tuning choices from hc_batch_autotune, or NULL for defaults.
 * A chunk's ToA span must fit 2^(64 - bits(n_chunks - 1)) ticks, else its
 * status is HC_ERR_RANGE. */
typedef struct hc_batch_plan hc_batch_plan;
typedef struct hc_batch_graph hc_batch_graph;

int hc_cluster_batch(const hc_hit* hits, const int64_t* offsets, int32_t n_chunks, const uint64_t* dts,
                     int32_t* labels, hc_features* features, int32_t* n_clusters, const hc_batch_plan* plan,
                     const hc_opts* opts);

/* Bytes of workspace hc_cluster_batch needs (opts->workspace may supply it). */
size_t hc_batch_workspace_size(const int64_t* offsets, int32_t n_chunks, const hc_batch_plan* plan,
                               const hc_opts* opts);

/* Autotuner: runs every candidate plan (sort tile size / neighbour reach, XCD
 * tile mapping, neighbour search variant) on this batch, rejects any candidate whose labels, features
 * or counts differ from the default plan's in a single bit, and returns the
 * fastest.  Uses labels/features/n_clusters as scratch (they end up holding
 * the result).  The choice is cached per (device, size class) for the process. */
int hc_batch_autotune(const hc_hit* hits, const int64_t* offsets, int32_t n_chunks, const uint64_t* dts,
                      int32_t* labels, hc_features* features, int32_t* n_clusters, const hc_opts* opts,
                      hc_batch_plan** out);
/* Human-readable plan (e.g. "disorder_hint=1024 sort_tile=2048 xcd_map=1
 * link=default time_ms=0.42"). */
int hc_batch_plan_describe(const hc_batch_plan* plan, char* buf, size_t cap);
void hc_batch_plan_destroy(hc_batch_plan* plan);

/* Capture the whole batch launch sequence (same arguments, fixed pointers) in
 * a HIP graph; hc_batch_graph_launch replays it on `stream` (a hipStream_t).
 * The graph owns its workspace; inputs may change between replays, sizes may
 * not. */
int hc_batch_graph_create(const hc_hit* hits, const int64_t* offsets, int32_t n_chunks, const uint64_t* dts,
                          int32_t* labels, hc_features* features, int32_t* n_clusters,
                          const hc_batch_plan* plan, const hc_opts* opts, hc_batch_graph** out);
int hc_batch_graph_launch(hc_batch_graph* graph, void* stream);
void hc_batch_graph_destroy(hc_batch_graph* graph);

/* ---- Served form: continuous batching of many detector streams ---------
 *
 * A request loop for detector chunks that arrive over time (the paper's
 * online setting: hits are read, clustered and handed on while the detector
 * keeps taking data, Sections 3 and 4).  Every detector stream owns an
 * hc_stream (device-resident open clusters, exact stitching across chunks)
 * on its own HIP stream and host worker thread, so the device work of
 * different streams overlaps.  A chunk is admitted when one of `max_slots`
 * slots is free and the device memory it needs (its hits and labels, plus the
 * growth of its stream's state) fits in `hbm_budget` beside everything the
 * server already holds; otherwise it waits, in arrival order per stream.
 * Chunks of a stream queued together share one push, and one slot, as long
 * as they fit in max_chunk_hits together (at most 16 chunks).
 *
 * Host buffers: hits[n] is copied to the device after admission and labels[n]
 * receives the chunk's final (stream-global) labels; both belong to the
 * caller and must stay valid until the chunk's completion is polled.  Pinned
 * memory (hipHostMalloc) makes the copies asynchronous DMA.
 * Every call is thread-safe; submissions to one stream must come in stream
 * order (one producer per stream). */
typedef struct hc_server hc_server;

typedef struct {
    uint32_t width, height;      /* sensor of every stream (0 => 256) */
    int32_t n_streams;           /* stream ids 0 .. n_streams - 1 (1..256) */
    int32_t max_slots;           /* pushes in device processing at once (0 => 2 * n_streams) */
    uint64_t dt;                 /* time window of the clusters, ticks */
    uint64_t max_disorder_ticks; /* t of every stream (see hc_stream_create) */
    uint64_t hbm_budget;         /* bytes of device memory the server may hold (0 => 16 GiB) */
    uint32_t disorder_hint;      /* positional displacement hint (0 => 4096) */
    uint32_t flags;              /* must be 0 */
    int32_t max_chunk_hits;      /* buffers are reserved up front for chunks this large (0 => 2^20) */
    int32_t reserved;            /* must be 0 */
} hc_server_config;

typedef struct {
    uint64_t tag;            /* caller's tag of the chunk */
    int32_t stream_id;
    int32_t status;          /* HC_OK, or why the chunk was rejected (labels then untouched) */
    int32_t n_hits;
    int32_t n_closed;        /* clusters closed by this chunk's push (0 if rejected) */
    uint64_t t_arrive_ns;    /* the caller's arrival stamp (hc_server_now_ns clock) */
    uint64_t t_admit_ns;     /* admitted: slot and memory granted */
    uint64_t t_processed_ns; /* device work done; closed clusters copied to the host */
    uint64_t t_final_ns;     /* every label of the chunk final and in labels[] */
} hc_completion;

typedef struct {
    int64_t submitted, completed, rejected, hits_completed;
    int64_t queued;            /* submitted chunks not yet admitted */
    int64_t pending_final;     /* processed chunks whose labels are not final yet */
    uint64_t hbm_budget, hbm_in_use, hbm_peak;
    int32_t max_slots, peak_slots_in_use;
    /* latency quantiles over all completed chunks, ns */
    uint64_t processing_p50, processing_p99, final_p50, final_p99;
    /* worker time summed over streams, ns: waiting for admission, copying
     * hits in and pushing, moving closed clusters out, copying final labels */
    uint64_t ns_admit_wait, ns_push, ns_drain, ns_final;
    int64_t pushes; /* device pushes (one push carries the chunks of a stream queued together) */
} hc_server_stats;

/* Monotonic clock (ns) for t_arrive stamps. */
uint64_t hc_server_now_ns(void);

/* Start the worker threads and per-stream state on the current device. */
int hc_server_create(const hc_server_config* cfg, hc_server** out);

/* Queue a chunk of stream `stream_id` (never blocks on the device).
 * Returns HC_ERR_ARG for a bad id or buffer, HC_ERR_BUDGET if a chunk of n
 * hits can never fit the budget, HC_ERR_BUSY after hc_server_destroy began. */
int hc_server_submit(hc_server* s, int32_t stream_id, const hc_hit* hits, int32_t n, int32_t* labels,
                     uint64_t tag, uint64_t t_arrive_ns);

/* End of stream `stream_id`: close all its open clusters once the chunks
 * queued before this call are processed (their labels then become final). */
int hc_server_flush(hc_server* s, int32_t stream_id);

/* Completed chunks (final labels or rejection), oldest first. */
int hc_server_poll(hc_server* s, hc_completion* out, int32_t cap, int32_t* n_out);

/* Features of closed clusters of one stream (stream-global labels), in
 * closing order; up to cap into out (caller's memory), *n_out written.
 * Records not read yet stay in host memory held by the server; reading them
 * as they come lets it reuse those host blocks (fresh host memory costs the
 * workers a page fault per 4 KiB, which limits a saturated server). */
int hc_server_closed(hc_server* s, int32_t stream_id, hc_features* out, int32_t cap, int32_t* n_out);

/* Wait until no chunk is queued or in device processing (chunks waiting for
 * finality may remain until more data or a flush); HC_ERR_BUSY on timeout. */
int hc_server_wait_idle(hc_server* s, int32_t timeout_ms);

int hc_server_stats_read(hc_server* s, hc_server_stats* out);

/* Stops the workers after the work already queued, frees all device state. */
void hc_server_destroy(hc_server* s);

/* Human-readable description of the last error on this thread. */
const char* hc_last_error(void);

/* Library version string. */
const char* hc_version(void);

/* ---- kernel timing (diagnostics) --------------------------------------
 * When enabled, every kernel the library launches is bracketed by HIP events
 * on the stream it runs on.  hc_timing_read reports, per kernel name, the
 * number of launches and the summed duration in milliseconds since the last
 * reset; it synchronises with the recorded events.  Not thread-safe: enable
 * it only in single-threaded measurement code. */
int hc_timing_enable(int on);
/* Restrict the timing to launches of one kernel (a name hc_timing_read
 * reports, e.g. "link"), so that the other launches carry no events; NULL or
 * "" times every kernel again.  Returns HC_OK. */
int hc_timing_select(const char* name);
int hc_timing_reset(void);
/* Writes up to cap entries; names are static strings owned by the library.
 * Returns the number of distinct kernels (may exceed cap), or < 0 on error. */
int hc_timing_read(const char** names, int64_t* launches, double* total_ms, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
