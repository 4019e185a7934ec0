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
 *                             clustering": sort by ToA, search the 8
 *                             neighbouring pixels plus the pixel itself for
 *                             the latest earlier hit, and join clusters with a
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
 *     share a workspace must be ordered by the caller (same stream).
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
    uint32_t flags;          /* reserved, 0 */
    void* workspace;         /* device scratch of >= hc_workspace_size bytes,
                                or NULL: the library then keeps a cached
                                per-device buffer (grown with hipMalloc) */
    size_t workspace_bytes;
    void* stream;            /* hipStream_t to run on; NULL = null stream */
} hc_opts;

enum {
    HC_OK = 0,
    HC_ERR_ARG = -1,       /* bad argument (NULL pointer, n < 0, bad size) */
    HC_ERR_RANGE = -2,     /* a hit has x >= width or y >= height */
    HC_ERR_WORKSPACE = -3, /* workspace smaller than hc_workspace_size */
    HC_ERR_DEVICE = -4,    /* HIP runtime error (see hc_last_error) */
    HC_ERR_DISORDER = -5,  /* stream: a hit violates the disorder contract */
    HC_ERR_OVERFLOW = -6,  /* more than 2^31 - 1 hits in one labelling */
    HC_ERR_BUDGET = -7,    /* server: request exceeds the memory budget */
    HC_ERR_BUSY = -8       /* server: no slot free */
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
 * toa_max + dt <= M - t.
 *
 * Labels are stream-global: the smallest global index (0-based position in
 * the concatenation of all pushed chunks) of the hit's cluster.  They are
 * written into each chunk's labels buffer as its clusters close, possibly
 * during a later push or the flush; a chunk is complete when its tag is
 * reported by hc_stream_poll.  At most 2^31 - 1 hits per stream.
 * A stream is single-producer; all its work runs on opts->stream. */
typedef struct hc_stream hc_stream;

/* opts: sensor size, disorder_hint (positional, for the sort), stream; the
 * workspace fields are ignored (the stream owns its device buffers). */
int hc_stream_create(const hc_opts* opts, uint64_t dt, uint64_t max_disorder_ticks, hc_stream** out);

/* Append n hits (device array).  labels: device int32[n] that the library
 * fills as the chunk's clusters close; it must stay valid until `tag` is
 * returned by hc_stream_poll.  Returns HC_ERR_DISORDER (chunk rejected,
 * stream unchanged) if a hit has toa <= M - t, HC_ERR_RANGE (rejected) if a
 * hit is off the sensor, HC_ERR_OVERFLOW past 2^31 - 1 hits.  Blocks until
 * the chunk has been processed on the device. */
int hc_stream_push(hc_stream* s, const hc_hit* hits, int32_t n, int32_t* labels, uint64_t tag);

/* Drain completion events into HOST buffers: up to cap tags of chunks whose
 * labels are all final (in completion order), and up to closed_cap features
 * of closed clusters (labels stream-global; ascending label within one push).
 * Entries beyond the caps stay queued for the next call. */
int hc_stream_poll(hc_stream* s, uint64_t* done_tags, int32_t cap, int32_t* n_done, hc_features* closed,
                   int32_t closed_cap, int32_t* n_closed);

/* Close every open cluster (end of stream); afterwards all pushed chunks are
 * complete. */
int hc_stream_flush(hc_stream* s);

void hc_stream_destroy(hc_stream* s);

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
int hc_timing_reset(void);
/* Writes up to cap entries; names are static strings owned by the library.
 * Returns the number of distinct kernels (may exceed cap), or < 0 on error. */
int hc_timing_read(const char** names, int64_t* launches, double* total_ms, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
