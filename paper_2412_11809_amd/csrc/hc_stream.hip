// Stream form: exact clustering of one detector's hit stream pushed in
// chunks, with clusters that straddle chunk borders stitched on the device.
//
// The paper fills buffers so that unsortedness never splits a cluster and
// then checks the borders (its buffer-filling algorithm and step 5 of its
// high-level GPU algorithm); its CPU pipeline keeps "open clusters" until
// they can no longer grow and then dispatches them (Section 3.3, Algorithm
// "processHit").  Here the open state is the set of hits whose cluster may
// still grow.  Every push appends the new chunk behind those hits (in global
// index order, so the smallest buffer position of a cluster is also its
// smallest global index), clusters the buffer with the plain path, and
// closes every cluster with toa_max + dt <= M - t (M = largest ToA pushed, t
// = the disorder bound: every later hit has toa > M - t, so it cannot join).
// Closed hits get their final stream-global label written into their chunk's
// buffer; closed clusters' features are queued for polling; the rest stays
// open (stable compaction).
#include <string.h>

#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "hc_device.h"

namespace hc {

struct StreamDev {
    unsigned long long chunk_max;  // largest ToA of the chunk being appended
    int32_t disorder;              // a hit at or below the watermark
    int32_t range;                 // a hit off the sensor
    int32_t n_keep;                // open hits after the push
    int32_t n_closed;              // clusters closed by the push
    int32_t n_clusters;            // clusters of the buffer (or an error status)
    int32_t pad_;
};

struct ChunkRec {
    int32_t* labels;  // caller's buffer for the chunk's labels
    int64_t base;     // global index of the chunk's first hit
    int32_t count;
    int32_t open;     // hits whose label is not final yet
};

constexpr int kCmpBlock = 2048;
constexpr int kCmpThreads = 256;

__device__ inline uint64_t sat_add_u64(uint64_t a, uint64_t b) { return ~0ull - a < b ? ~0ull : a + b; }

__global__ __launch_bounds__(256) void k_stream_append(const hc_hit* __restrict__ in, int n, hc_hit* buf,
                                                       int32_t* gidx, int32_t* cslot, int n_open, int32_t base,
                                                       int slot, uint64_t wmark, int has_wmark, uint32_t W,
                                                       uint32_t H, StreamDev* sd)
{
    __shared__ uint64_t red[256 / kWave];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t mx = 0;
    if (i < n) {
        const hc_hit h = in[i];
        buf[n_open + i] = h;
        gidx[n_open + i] = base + i;
        cslot[n_open + i] = slot;
        mx = h.toa;
        if (has_wmark && h.toa <= wmark) atomicOr(&sd->disorder, 1);
        if (h.x >= W || h.y >= H) atomicOr(&sd->range, 1);
    }
    mx = block_max_u64<256>(mx, red);
    if (threadIdx.x == 0) atomicMax(&sd->chunk_max, (unsigned long long)mx);
}

// A hit is final when its cluster is closed: write its stream-global label
// into its chunk's buffer.  keep[i] = 1 for hits that stay open.
__global__ void k_stream_close_hits(int n_all, const int32_t* __restrict__ lab, const Work w,
                                    const int32_t* __restrict__ gidx, const int32_t* __restrict__ cslot,
                                    ChunkRec* chunks, uint64_t wmark, int has_wmark, uint64_t dt, int flush,
                                    uint8_t* keep)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    bool closed = false;
    int32_t slot = -1;
    if (i < n_all) {
        const int32_t r = lab[i];
        closed = flush || (has_wmark && sat_add_u64(w.slots[root_rank(w, 0, 0, r)].toa_max, dt) <= wmark);
        if (closed) {
            slot = cslot[i];
            ChunkRec* ch = chunks + slot;
            ch->labels[gidx[i] - ch->base] = gidx[r];
        }
        keep[i] = closed ? 0 : 1;
    }
    // one decrement per chunk per wave (a wave's hits mostly share a chunk),
    // not one atomic per hit on the same counter
    unsigned long long pending = __ballot(closed);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int32_t s = __shfl(slot, leader, kWave);
        const unsigned long long same = __ballot(closed && slot == s);
        if (lane == leader) atomicSub(&chunks[s].open, (int32_t)__popcll(same));
        pending &= ~same;
    }
}

// flag[k] = 1 for clusters (feature rows, ascending label) that are closed
__global__ void k_stream_close_feats(const hc_features* __restrict__ f, int cap, const StreamDev* sd, uint64_t wmark,
                                     int has_wmark, uint64_t dt, int flush, uint8_t* flag)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cap) return;
    const int K = sd->n_clusters;
    flag[k] = (k < K && (flush || (has_wmark && sat_add_u64(f[k].toa_max, dt) <= wmark))) ? 1 : 0;
}

// Stable compaction by flag, in three steps: per-block counts, one
// work-group scan of the counts, scatter.
__global__ __launch_bounds__(kCmpThreads) void k_flag_count(const uint8_t* __restrict__ flag, int n, uint32_t* counts)
{
    __shared__ uint32_t wsum[kCmpThreads / kWave];
    const int64_t b0 = (int64_t)blockIdx.x * kCmpBlock;
    uint32_t c = 0;
    for (int q = 0; q < kCmpBlock / kCmpThreads; q++) {
        const int64_t i = b0 + q * kCmpThreads + threadIdx.x;
        c += (i < n && flag[i]) ? 1u : 0u;
    }
    uint32_t total;
    block_exclusive_scan<kCmpThreads>(c, wsum, &total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_flag_scan(uint32_t* counts, int nb, int32_t* total_out)
{
    __shared__ uint32_t wsum[1024 / kWave];
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < nb ? counts[i] : 0u;
        uint32_t total;
        const uint32_t e = block_exclusive_scan<1024>(v, wsum, &total);
        if (i < nb) counts[i] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = (int32_t)carry;
}

// position of every flagged item of this block (PER consecutive items per thread)
template <class F>
__device__ inline void flag_scatter(const uint8_t* __restrict__ flag, int n, const uint32_t* offs, F&& emit)
{
    __shared__ uint32_t wsum[kCmpThreads / kWave];
    constexpr int PER = kCmpBlock / kCmpThreads;
    const int64_t i0 = (int64_t)blockIdx.x * kCmpBlock + (int64_t)threadIdx.x * PER;
    uint32_t bits = 0;
#pragma unroll
    for (int q = 0; q < PER; q++)
        if (i0 + q < n && flag[i0 + q]) bits |= 1u << q;
    uint64_t pos = (uint64_t)offs[blockIdx.x] + block_exclusive_scan<kCmpThreads>(__popc(bits), wsum, nullptr);
#pragma unroll
    for (int q = 0; q < PER; q++)
        if (bits & (1u << q)) emit(i0 + q, pos++);
}

__global__ __launch_bounds__(kCmpThreads) void k_scatter_open(const uint8_t* __restrict__ flag, int n,
                                                              const uint32_t* offs, const hc_hit* __restrict__ sb,
                                                              const int32_t* __restrict__ sg,
                                                              const int32_t* __restrict__ sc, hc_hit* db,
                                                              int32_t* dg, int32_t* dc)
{
    flag_scatter(flag, n, offs, [&](int64_t i, uint64_t p) {
        db[p] = sb[i];
        dg[p] = sg[i];
        dc[p] = sc[i];
    });
}

__global__ __launch_bounds__(kCmpThreads) void k_scatter_feats(const uint8_t* __restrict__ flag, int n,
                                                               const uint32_t* offs,
                                                               const hc_features* __restrict__ f,
                                                               const int32_t* __restrict__ gidx, hc_features* q,
                                                               int64_t q_base)
{
    flag_scatter(flag, n, offs, [&](int64_t k, uint64_t p) {
        hc_features r = f[k];
        r.label = gidx[r.label];
        q[q_base + p] = r;
    });
}

}  // namespace hc

// ===================================================================== host
using namespace hc;

namespace {

template <class T>
int dev_alloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    return e == hipSuccess ? HC_OK : set_device_error(e, "hipMalloc(stream)");
}

struct ChunkHost {
    uint64_t tag;
    bool active;
};

}  // namespace

struct hc_stream {
    hipStream_t s = nullptr;
    uint32_t W = 256, H = 256, D = 4096;
    int32_t link_mode = 0;
    uint64_t dt = 0, tdis = 0;
    // open buffer (ping-pong) and per-push scratch, capacity `cap` hits
    int64_t cap = 0;
    int cur = 0;
    hc_hit* buf[2] = {nullptr, nullptr};
    int32_t* gidx[2] = {nullptr, nullptr};
    int32_t* cslot[2] = {nullptr, nullptr};
    uint8_t* flags = nullptr;
    int32_t* lab = nullptr;
    hc_features* feats = nullptr;
    uint32_t* counts = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // closed-cluster queue (device)
    hc_features* queue = nullptr;
    int64_t q_cap = 0, q_count = 0;
    // chunk table
    ChunkRec* chunks_dev = nullptr;
    ChunkRec* chunks_pin = nullptr;  // pinned mirror
    int chunk_cap = 0;
    std::vector<ChunkHost> chunks;
    std::deque<uint64_t> done;
    // small device state + pinned mirror
    StreamDev* sd = nullptr;
    StreamDev* sd_pin = nullptr;
    int64_t n_open = 0, next_g = 0;
    uint64_t M = 0;
    bool has_M = false;
    // after a flush every later hit must lie more than dt after every flushed
    // hit (toa > floor = M + dt), so no cluster spans the flush
    uint64_t floor = 0;
    bool has_floor = false;
    bool failed = false;
};

static void free_all(hc_stream* st)
{
    for (int b = 0; b < 2; b++) {
        (void)hipFree(st->buf[b]);
        (void)hipFree(st->gidx[b]);
        (void)hipFree(st->cslot[b]);
    }
    (void)hipFree(st->flags);
    (void)hipFree(st->lab);
    (void)hipFree(st->feats);
    (void)hipFree(st->counts);
    (void)hipFree(st->ws);
    (void)hipFree(st->queue);
    (void)hipFree(st->chunks_dev);
    (void)hipFree(st->sd);
    (void)hipHostFree(st->chunks_pin);
    (void)hipHostFree(st->sd_pin);
}

static uint32_t sort_hint(const hc_stream* st, int64_t n_open)
{
    // the open hits precede the chunk in the buffer; a chunk hit can move up
    // to n_open places plus the chunk's own disorder
    const int64_t h = (int64_t)st->D + n_open;
    return (uint32_t)(h > 0x7FFFFFFF ? 0x7FFFFFFF : h);
}

// Grow the per-push buffers to hold n_all hits, keeping the open hits.
static int ensure_capacity(hc_stream* st, int64_t n_all)
{
    hipError_t e;
    if (n_all > st->cap) {
        int64_t nc = st->cap * 2 > n_all ? st->cap * 2 : n_all;
        if (nc < 4096) nc = 4096;
        if ((e = hipStreamSynchronize(st->s)) != hipSuccess) return set_device_error(e, "hipStreamSynchronize");
        hc_hit* nb[2];
        int32_t* ng[2];
        int32_t* ncs[2];
        int rc = HC_OK;
        for (int b = 0; b < 2 && rc == HC_OK; b++) {
            if ((rc = dev_alloc(&nb[b], nc)) != HC_OK) break;
            if ((rc = dev_alloc(&ng[b], nc)) != HC_OK) break;
            rc = dev_alloc(&ncs[b], nc);
        }
        if (rc != HC_OK) return rc;
        if (st->n_open > 0) {
            (void)hipMemcpy(nb[0], st->buf[st->cur], sizeof(hc_hit) * st->n_open, hipMemcpyDeviceToDevice);
            (void)hipMemcpy(ng[0], st->gidx[st->cur], 4 * st->n_open, hipMemcpyDeviceToDevice);
            (void)hipMemcpy(ncs[0], st->cslot[st->cur], 4 * st->n_open, hipMemcpyDeviceToDevice);
        }
        for (int b = 0; b < 2; b++) {
            (void)hipFree(st->buf[b]);
            (void)hipFree(st->gidx[b]);
            (void)hipFree(st->cslot[b]);
            st->buf[b] = nb[b];
            st->gidx[b] = ng[b];
            st->cslot[b] = ncs[b];
        }
        st->cur = 0;
        (void)hipFree(st->flags);
        (void)hipFree(st->lab);
        (void)hipFree(st->feats);
        (void)hipFree(st->counts);
        if ((rc = dev_alloc(&st->flags, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->lab, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->feats, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->counts, (nc + kCmpBlock - 1) / kCmpBlock + 1)) != HC_OK) return rc;
        st->cap = nc;
    }
    const size_t need = plan_workspace(n_all, st->W, st->H, sort_hint(st, st->n_open), nullptr, nullptr);
    if (need > st->ws_bytes) {
        if ((e = hipStreamSynchronize(st->s)) != hipSuccess) return set_device_error(e, "hipStreamSynchronize");
        (void)hipFree(st->ws);
        st->ws = nullptr;
        st->ws_bytes = 0;
        const size_t nb = need + need / 4;
        if ((e = hipMalloc(&st->ws, nb)) != hipSuccess) return set_device_error(e, "hipMalloc(stream workspace)");
        st->ws_bytes = nb;
    }
    if (st->q_count + n_all > st->q_cap) {
        if ((e = hipStreamSynchronize(st->s)) != hipSuccess) return set_device_error(e, "hipStreamSynchronize");
        int64_t nq = st->q_cap * 2 > st->q_count + n_all ? st->q_cap * 2 : st->q_count + n_all;
        hc_features* q;
        int rc = dev_alloc(&q, nq);
        if (rc != HC_OK) return rc;
        if (st->q_count) (void)hipMemcpy(q, st->queue, sizeof(hc_features) * st->q_count, hipMemcpyDeviceToDevice);
        (void)hipFree(st->queue);
        st->queue = q;
        st->q_cap = nq;
    }
    return HC_OK;
}

// Device bytes a stream holds with buffers for `cap` hits, a workspace of
// `ws` bytes, a closed-cluster queue of `q` records and `chunks` chunk slots.
static size_t footprint(int64_t cap, size_t ws, int64_t q, int chunks)
{
    const size_t per_hit = 2 * (sizeof(hc_hit) + 4 + 4) + 1 + 4 + sizeof(hc_features);
    return (size_t)cap * per_hit + 4 * (size_t)((cap + kCmpBlock - 1) / kCmpBlock + 1) + ws +
           sizeof(hc_features) * (size_t)q + sizeof(ChunkRec) * (size_t)chunks + sizeof(StreamDev);
}

static int grow_chunks(hc_stream* st)
{
    hipError_t e;
    const int nc = st->chunk_cap ? st->chunk_cap * 2 : 64;
    if ((e = hipStreamSynchronize(st->s)) != hipSuccess) return set_device_error(e, "hipStreamSynchronize");
    ChunkRec* d;
    ChunkRec* p;
    int rc = dev_alloc(&d, nc);
    if (rc != HC_OK) return rc;
    if ((e = hipHostMalloc((void**)&p, sizeof(ChunkRec) * nc, hipHostMallocDefault)) != hipSuccess)
        return set_device_error(e, "hipHostMalloc");
    if (st->chunk_cap) {
        (void)hipMemcpy(d, st->chunks_dev, sizeof(ChunkRec) * st->chunk_cap, hipMemcpyDeviceToDevice);
        ::memcpy(p, st->chunks_pin, sizeof(ChunkRec) * st->chunk_cap);
    }
    (void)hipFree(st->chunks_dev);
    (void)hipHostFree(st->chunks_pin);
    st->chunks_dev = d;
    st->chunks_pin = p;
    st->chunks.resize(nc, ChunkHost{0, false});
    st->chunk_cap = nc;
    return HC_OK;
}

// Cluster the buffer (open hits + new chunk), close what can be closed,
// compact the rest.  has_wmark: every later hit has toa > wmark (without a
// watermark -- the largest ToA is still below t -- nothing closes).
static int process(hc_stream* st, int64_t n_all, uint64_t wmark, bool has_wmark, int flush)
{
    hipError_t e;
    const int n = (int)n_all;
    Work w;
    plan_workspace(n_all, st->W, st->H, sort_hint(st, st->n_open), &w, (char*)st->ws);
    w.dt = st->dt;
    w.link_mode = st->link_mode;
    int rc = enqueue_cluster(st->buf[st->cur], w, st->lab, st->feats, &st->sd->n_clusters, st->s);
    if (rc != HC_OK) return rc;
    const int blocks = (n + 255) / 256;
    TimedLaunch tl("stream_close", st->s);  // the closing and compaction kernels below, together
    const int nb = (n + kCmpBlock - 1) / kCmpBlock;
    const int nxt = 1 - st->cur;
    hipLaunchKernelGGL(k_stream_close_hits, dim3(blocks), dim3(256), 0, st->s, n, st->lab, w,
                       st->gidx[st->cur], st->cslot[st->cur], st->chunks_dev, wmark, has_wmark ? 1 : 0, st->dt, flush,
                       st->flags);
    hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, n, st->counts);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st->s, st->counts, nb, &st->sd->n_keep);
    hipLaunchKernelGGL(k_scatter_open, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, n, st->counts,
                       st->buf[st->cur], st->gidx[st->cur], st->cslot[st->cur], st->buf[nxt], st->gidx[nxt],
                       st->cslot[nxt]);
    hipLaunchKernelGGL(k_stream_close_feats, dim3(blocks), dim3(256), 0, st->s, st->feats, n, st->sd, wmark,
                       has_wmark ? 1 : 0, st->dt, flush, st->flags);
    hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, n, st->counts);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st->s, st->counts, nb, &st->sd->n_closed);
    hipLaunchKernelGGL(k_scatter_feats, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, n, st->counts,
                       st->feats, st->gidx[st->cur], st->queue, st->q_count);
    if ((e = hipGetLastError()) != hipSuccess) return set_device_error(e, "stream close");
    if ((e = hipMemcpyAsync(st->sd_pin, st->sd, sizeof(StreamDev), hipMemcpyDeviceToHost, st->s)) != hipSuccess ||
        (e = hipMemcpyAsync(st->chunks_pin, st->chunks_dev, sizeof(ChunkRec) * st->chunk_cap,
                            hipMemcpyDeviceToHost, st->s)) != hipSuccess ||
        (e = hipStreamSynchronize(st->s)) != hipSuccess)
        return set_device_error(e, "stream readback");
    if (st->sd_pin->n_clusters < 0) {
        st->failed = true;
        return set_error(HC_ERR_DEVICE, "stream: internal clustering error");
    }
    st->n_open = st->sd_pin->n_keep;
    st->cur = nxt;
    st->q_count += st->sd_pin->n_closed;
    for (int c = 0; c < st->chunk_cap; c++) {
        if (st->chunks[c].active && st->chunks_pin[c].open == 0) {
            st->chunks[c].active = false;
            st->done.push_back(st->chunks[c].tag);
        }
    }
    return HC_OK;
}

namespace hc {

size_t stream_device_bytes(const hc_stream* st) { return footprint(st->cap, st->ws_bytes, st->q_cap, st->chunk_cap); }

// What the stream will hold after pushing a chunk of n hits (the growth rules
// of ensure_capacity and grow_chunks); *transient: bytes of old buffers that
// are alive together with their replacements while growing.
size_t stream_bytes_after_push(const hc_stream* st, int64_t n, size_t* transient)
{
    const int64_t n_all = st->n_open + n;
    int64_t cap = st->cap;
    size_t tr = 0;
    if (n_all > cap) {
        cap = st->cap * 2 > n_all ? st->cap * 2 : n_all;
        if (cap < 4096) cap = 4096;
        tr += footprint(st->cap, 0, 0, 0);
    }
    const size_t need = plan_workspace(n_all, st->W, st->H, sort_hint(st, st->n_open), nullptr, nullptr);
    const size_t ws = need > st->ws_bytes ? need + need / 4 : st->ws_bytes;
    int64_t q = st->q_cap;
    if (st->q_count + n_all > q) {
        q = st->q_cap * 2 > st->q_count + n_all ? st->q_cap * 2 : st->q_count + n_all;
        tr += sizeof(hc_features) * (size_t)st->q_cap;
    }
    int chunks = st->chunk_cap;
    bool free_slot = false;
    for (int c = 0; c < st->chunk_cap && !free_slot; c++) free_slot = !st->chunks[c].active;
    if (!free_slot) {
        chunks = st->chunk_cap ? st->chunk_cap * 2 : 64;
        tr += sizeof(ChunkRec) * (size_t)st->chunk_cap;
    }
    if (transient) *transient = tr;
    return footprint(cap, ws, q, chunks);
}

int64_t stream_open_hits(const hc_stream* st) { return st->n_open; }

}  // namespace hc

extern "C" {

int hc_stream_create(const hc_opts* opts, uint64_t dt, uint64_t max_disorder_ticks, hc_stream** out)
{
    if (!out) return set_error(HC_ERR_ARG, "out is NULL");
    *out = nullptr;
    hc_stream* st = new hc_stream();
    st->W = opts && opts->width ? opts->width : 256;
    st->H = opts && opts->height ? opts->height : 256;
    st->D = opts && opts->disorder_hint ? opts->disorder_hint : 4096;
    st->s = opts ? (hipStream_t)opts->stream : nullptr;
    st->dt = dt;
    st->tdis = max_disorder_ticks;
    st->link_mode = link_mode_of(opts);
    if (st->W > 65535 || st->H > 65535 || (opts && !link_flags_valid(opts->flags))) {
        delete st;
        return set_error(HC_ERR_ARG, "bad stream options");
    }
    hipError_t e;
    int rc = dev_alloc(&st->sd, 1);
    if (rc == HC_OK && (e = hipHostMalloc((void**)&st->sd_pin, sizeof(StreamDev), hipHostMallocDefault)) != hipSuccess)
        rc = set_device_error(e, "hipHostMalloc");
    if (rc == HC_OK) rc = grow_chunks(st);
    if (rc != HC_OK) {
        free_all(st);
        delete st;
        return rc;
    }
    *out = st;
    return HC_OK;
}

int hc_stream_push(hc_stream* st, const hc_hit* hits, int32_t n, int32_t* labels, uint64_t tag)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    if (n < 0 || (n > 0 && (!hits || !labels))) return set_error(HC_ERR_ARG, "bad chunk arguments");
    if (st->next_g + n > 0x7FFFFFFF) return set_error(HC_ERR_OVERFLOW, "more than 2^31 - 1 hits in the stream");
    if (n == 0) {
        st->done.push_back(tag);
        return HC_OK;
    }
    const int64_t n_all = st->n_open + n;
    int rc = ensure_capacity(st, n_all);
    if (rc != HC_OK) return rc;
    int slot = -1;
    for (int c = 0; c < st->chunk_cap; c++)
        if (!st->chunks[c].active) {
            slot = c;
            break;
        }
    if (slot < 0) {
        if ((rc = grow_chunks(st)) != HC_OK) return rc;
        for (int c = 0; c < st->chunk_cap; c++)
            if (!st->chunks[c].active) {
                slot = c;
                break;
            }
    }
    // append and validate (a rejected chunk leaves the open state untouched:
    // only buffer positions beyond n_open are written)
    hipError_t e;
    // a hit is rejected when toa <= M - t (the t-ordered contract; no bound
    // while M < t) or, after a flush, toa <= floor
    const bool has_w = st->has_M && st->M >= st->tdis;
    uint64_t wmark = has_w ? st->M - st->tdis : 0;
    if (st->has_floor && (!has_w || st->floor > wmark)) wmark = st->floor;
    const bool reject_below = has_w || st->has_floor;
    ::memset(st->sd_pin, 0, sizeof(StreamDev));
    if ((e = hipMemcpyAsync(st->sd, st->sd_pin, sizeof(StreamDev), hipMemcpyHostToDevice, st->s)) != hipSuccess)
        return set_device_error(e, "stream reset");
    {
        TimedLaunch tl("stream_append", st->s);
        hipLaunchKernelGGL(k_stream_append, dim3((n + 255) / 256), dim3(256), 0, st->s, hits, n,
                           st->buf[st->cur], st->gidx[st->cur], st->cslot[st->cur], (int)st->n_open,
                           (int32_t)st->next_g, slot, wmark, reject_below ? 1 : 0, st->W, st->H, st->sd);
    }
    if ((e = hipGetLastError()) != hipSuccess) return set_device_error(e, "stream append");
    if ((e = hipMemcpyAsync(st->sd_pin, st->sd, sizeof(StreamDev), hipMemcpyDeviceToHost, st->s)) != hipSuccess ||
        (e = hipStreamSynchronize(st->s)) != hipSuccess)
        return set_device_error(e, "stream append readback");
    if (st->sd_pin->range) return set_error(HC_ERR_RANGE, "stream chunk has a hit off the sensor");
    if (st->sd_pin->disorder)
        return set_error(HC_ERR_DISORDER, "stream chunk has a hit at or below the disorder watermark");
    const uint64_t cmax = st->sd_pin->chunk_max;
    // register the chunk
    st->chunks[slot] = ChunkHost{tag, true};
    st->chunks_pin[slot] = ChunkRec{labels, st->next_g, n, n};
    if ((e = hipMemcpyAsync(st->chunks_dev + slot, st->chunks_pin + slot, sizeof(ChunkRec), hipMemcpyHostToDevice,
                            st->s)) != hipSuccess)
        return set_device_error(e, "stream chunk table");
    const uint64_t M = st->has_M ? (cmax > st->M ? cmax : st->M) : cmax;
    rc = process(st, n_all, M >= st->tdis ? M - st->tdis : 0, M >= st->tdis, 0);
    if (rc != HC_OK) return rc;
    st->next_g += n;
    st->M = M;
    st->has_M = true;
    return HC_OK;
}

int hc_stream_reserve(hc_stream* st, int32_t max_chunk)
{
    if (!st || max_chunk < 0) return set_error(HC_ERR_ARG, "bad stream or size");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    const int64_t margin = max_chunk / 4 + 4096;  // open hits carried between pushes
    const int64_t n_all = (int64_t)max_chunk + (st->n_open > margin ? st->n_open : margin);
    // size the workspace for the sort hint a push with `margin` open hits uses
    const int64_t keep = st->n_open;
    st->n_open = st->n_open > margin ? st->n_open : margin;
    const size_t need = plan_workspace(n_all, st->W, st->H, sort_hint(st, st->n_open), nullptr, nullptr);
    st->n_open = keep;
    int rc = ensure_capacity(st, n_all);
    if (rc != HC_OK) return rc;
    if (need > st->ws_bytes) {
        hipError_t e;
        if ((e = hipStreamSynchronize(st->s)) != hipSuccess) return set_device_error(e, "hipStreamSynchronize");
        (void)hipFree(st->ws);
        st->ws = nullptr;
        st->ws_bytes = 0;
        if ((e = hipMalloc(&st->ws, need)) != hipSuccess) return set_device_error(e, "hipMalloc(stream workspace)");
        st->ws_bytes = need;
    }
    return HC_OK;
}

int64_t hc_stream_open_hits(const hc_stream* st) { return st ? st->n_open : -1; }

int hc_stream_flush(hc_stream* st)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    if (st->has_M) {
        st->floor = ~0ull - st->M < st->dt ? ~0ull : st->M + st->dt;
        st->has_floor = true;
    }
    if (st->n_open == 0) return HC_OK;
    int rc = ensure_capacity(st, st->n_open);
    if (rc != HC_OK) return rc;
    return process(st, st->n_open, 0, false, 1);
}

int hc_stream_poll(hc_stream* st, uint64_t* done_tags, int32_t cap, int32_t* n_done, hc_features* closed,
                   int32_t closed_cap, int32_t* n_closed)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    int32_t nd = 0;
    while (nd < cap && !st->done.empty() && done_tags) {
        done_tags[nd++] = st->done.front();
        st->done.pop_front();
    }
    if (n_done) *n_done = nd;
    int32_t nc = 0;
    if (closed && closed_cap > 0 && st->q_count > 0) {
        nc = (int32_t)(st->q_count < closed_cap ? st->q_count : closed_cap);
        hipError_t e = hipMemcpyAsync(closed, st->queue, sizeof(hc_features) * nc, hipMemcpyDeviceToHost, st->s);
        // move the rest to the front in pieces of nc records (never overlapping)
        for (int64_t at = nc; e == hipSuccess && at < st->q_count; at += nc) {
            const int64_t len = (st->q_count - at) < nc ? (st->q_count - at) : nc;
            e = hipMemcpyAsync(st->queue + (at - nc), st->queue + at, sizeof(hc_features) * len,
                               hipMemcpyDeviceToDevice, st->s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st->s);
        if (e != hipSuccess) return set_device_error(e, "stream poll");
        st->q_count -= nc;
    }
    if (n_closed) *n_closed = nc;
    return HC_OK;
}

void hc_stream_destroy(hc_stream* st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->s);
    free_all(st);
    delete st;
}

}  // extern "C"
