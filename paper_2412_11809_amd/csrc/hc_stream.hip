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
// buffer; closed clusters' features go to a ring of records for polling; the
// rest stays open (stable compaction).
//
// Pushes are asynchronous: the stream's state (open-hit count, next global
// index, M, the closed-feature ring's tail) lives in device memory, a commit
// kernel accepts or rejects each chunk on the device, and the clustering
// kernels read their hit count from there (the host sizes the grids with an
// upper bound).  After each push a pinned copy of that state and of the
// chunk table is taken; the host reads it once the push's event completes.
#include <string.h>

#include <deque>
#include <string>
#include <vector>

#include "hc_device.h"

namespace hc {

struct StreamDev {
    // across pushes
    int32_t n_open;               // open hits at the front of the current buffer
    int32_t next_g;               // global index of the next accepted hit
    unsigned long long M;         // largest accepted ToA (valid when has_M)
    unsigned long long floor;     // after a flush, later hits need toa > floor
    int32_t has_M, has_floor;
    long long q_tail;             // closed-feature records written so far (ring slot q_tail % q_cap)
    // the current push
    unsigned long long chunk_max; // largest ToA of the chunk being appended
    int32_t disorder, range;      // raised by the chunk's hits
    int32_t n_all;                // hits the push clusters: the open ones, plus the chunk if accepted
    int32_t verdict;              // HC_OK, or why the chunk was rejected
    int32_t n_closed;             // clusters closed by the push
    int32_t n_clusters;           // clusters of the buffer (or an error status)
    unsigned long long wmark;     // closing watermark of the push (valid when has_wmark)
    int32_t has_wmark;
    int32_t bad_id;               // a caller-supplied id of the chunk is negative
};

struct ChunkRec {
    int32_t* labels;  // caller's buffer for the chunk's labels
    int64_t base;     // global index of the chunk's first hit (-1: rejected)
    int32_t count;
    int32_t open;     // hits whose label is not final yet
};

constexpr int kCmpBlock = 2048;
constexpr int kCmpThreads = 256;

__device__ inline uint64_t sat_add_u64(uint64_t a, uint64_t b) { return ~0ull - a < b ? ~0ull : a + b; }

// Copy the chunk behind the open hits and check it against the stream's
// contract: every hit on the sensor, and above the watermark M - t (once
// M >= t) and, after a flush, above the floor.
__global__ __launch_bounds__(256) void k_stream_append(const hc_hit* __restrict__ in,
                                                       const int32_t* __restrict__ in_ids, int n, hc_hit* buf,
                                                       int32_t* gidx, int32_t* ids, int32_t* cslot, int slot,
                                                       StreamDev* sd, uint64_t tdis, uint32_t W, uint32_t H)
{
    __shared__ uint64_t red[256 / kWave];
    const int n_open = sd->n_open;
    const int32_t base = sd->next_g;
    const bool has_w = sd->has_M && sd->M >= tdis;
    uint64_t thr = has_w ? sd->M - tdis : 0;
    bool has_thr = has_w;
    if (sd->has_floor) {
        if (!has_thr || sd->floor > thr) thr = sd->floor;
        has_thr = true;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t mx = 0;
    if (i < n) {
        const hc_hit h = in[i];
        buf[n_open + i] = h;
        gidx[n_open + i] = base + i;
        cslot[n_open + i] = slot;
        if (ids) {
            const int32_t id = in_ids ? in_ids[i] : base + i;
            ids[n_open + i] = id;
            if (id < 0) atomicOr(&sd->bad_id, 1);
        }
        mx = h.toa;
        if (has_thr && h.toa <= thr) atomicOr(&sd->disorder, 1);
        if (h.x >= W || h.y >= H) atomicOr(&sd->range, 1);
    }
    mx = block_max_u64<256>(mx, red);
    if (threadIdx.x == 0) atomicMax(&sd->chunk_max, (unsigned long long)mx);
}

// Accept or reject the appended chunk (one thread): an accepted chunk is
// registered in the chunk table and joins the clustered hits, M advances and
// the closing watermark follows; a rejected one is left out (its hits sit
// beyond n_all), so the push only re-clusters the open hits and closes
// nothing new.  A flush clusters the open hits, closes all of them and sets
// the floor M + dt for whatever is pushed later.
__global__ void k_stream_commit(StreamDev* sd, ChunkRec* chunks, int slot, int32_t* labels, int n, uint64_t tdis,
                                uint64_t dt, int flush)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    StreamDev& d = *sd;
    d.n_closed = 0;
    d.n_clusters = 0;  // set by the clustering, which a push with nothing to cluster skips
    if (flush) {
        d.verdict = HC_OK;
        d.n_all = d.n_open;
        d.has_wmark = 0;
        d.wmark = 0;
        if (d.has_M) {
            d.floor = sat_add_u64(d.M, dt);
            d.has_floor = 1;
        }
        return;
    }
    const int v = d.bad_id ? HC_ERR_ARG : d.range ? HC_ERR_RANGE : d.disorder ? HC_ERR_DISORDER : HC_OK;
    d.verdict = v;
    if (v == HC_OK) {
        chunks[slot] = ChunkRec{labels, (int64_t)d.next_g, n, n};
        d.n_all = d.n_open + n;
        d.next_g += n;
        d.M = d.has_M ? (d.chunk_max > d.M ? d.chunk_max : d.M) : d.chunk_max;
        d.has_M = 1;
    } else {
        chunks[slot] = ChunkRec{labels, -1, n, 0};
        d.n_all = d.n_open;
    }
    d.has_wmark = d.has_M && d.M >= tdis;
    d.wmark = d.has_wmark ? d.M - tdis : 0;
}

// End of a push: advance the ring's tail, clear the chunk flags.
__global__ void k_stream_end(StreamDev* sd)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sd->q_tail += sd->n_closed;
    sd->chunk_max = 0;
    sd->disorder = 0;
    sd->range = 0;
    sd->bad_id = 0;
}

__global__ void k_stream_set_qtail(StreamDev* sd, long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) sd->q_tail = v;
}

// With caller-supplied ids a cluster's label is its smallest id: reduced per
// cluster (feature row) over all clustered hits before the closing.
__global__ void k_stream_idmin_init(int32_t* cmin, const StreamDev* sd)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < sd->n_all) cmin[k] = 0x7FFFFFFF;
}

__global__ void k_stream_idmin(const int32_t* __restrict__ lab, const Work w, const int32_t* __restrict__ ids,
                               const StreamDev* sd, int32_t* cmin)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sd->n_all || sd->n_clusters < 0) return;
    const int32_t r = lab[i];
    if (r < 0 || r > i) return;  // reported by the closing kernel
    atomicMin(&cmin[root_rank(w, 0, 0, r)], ids[i]);
}

// A hit is final when its cluster is closed: write its stream-global label
// into its chunk's buffer.  keep[i] = 1 for hits that stay open.  Every chunk
// counts its hits whose labels are not final yet; the decrements go through
// a small per-work-group table in LDS (a work-group's hits mostly come from
// one or two chunks), one global atomic per chunk and work-group, since
// atomics on one address from every wave serialise in the L2.
constexpr int kCloseThreads = 256;
constexpr int kCloseBlock = 2048;
constexpr int kCloseSlots = 8;

__global__ __launch_bounds__(kCloseThreads) void k_stream_close_hits(const int32_t* __restrict__ lab, const Work w,
                                                                     const int32_t* __restrict__ gidx,
                                                                     const int32_t* __restrict__ cslot,
                                                                     const int32_t* __restrict__ cmin,
                                                                     ChunkRec* chunks, const StreamDev* sd,
                                                                     uint64_t dt, int flush, uint8_t* keep)
{
    __shared__ int32_t s_slot[kCloseSlots];
    __shared__ int32_t s_cnt[kCloseSlots];
    const int n_all = sd->n_all;
    if (sd->n_clusters < 0) return;  // the clustering failed; the host reports it
    if ((int64_t)blockIdx.x * kCloseBlock >= n_all) return;
    if (threadIdx.x < kCloseSlots) {
        s_slot[threadIdx.x] = -1;
        s_cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    const bool has_wmark = sd->has_wmark;
    const uint64_t wmark = sd->wmark;
    const int lane = threadIdx.x & (kWave - 1);
    for (int q = 0; q < kCloseBlock / kCloseThreads; q++) {
        const int64_t i = (int64_t)blockIdx.x * kCloseBlock + q * kCloseThreads + threadIdx.x;
        bool closed = false;
        int32_t slot = -1;
        if (i < n_all) {
            int32_t r = lab[i];
            if (r < 0 || r > i) {
                atomicOr(&w.status->err_internal, 1);
                r = (int32_t)i;
            }
            const uint32_t rank = root_rank(w, 0, 0, r);
            closed = flush || (has_wmark && sat_add_u64(w.slots[rank].toa_max, dt) <= wmark);
            if (closed) {
                slot = cslot[i];
                ChunkRec* ch = chunks + slot;
                ch->labels[gidx[i] - ch->base] = cmin ? cmin[rank] : gidx[r];
            }
            keep[i] = closed ? 0 : 1;
        }
        // one count per chunk per wave, added into the work-group's table
        unsigned long long pending = __ballot(closed);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int32_t sl = __shfl(slot, leader, kWave);
            const unsigned long long same = __ballot(closed && slot == sl);
            if (lane == leader) {
                const int32_t c = (int32_t)__popcll(same);
                int e = -1;
                for (int k = 0; k < kCloseSlots && e < 0; k++) {
                    const int32_t old = atomicCAS(&s_slot[k], -1, sl);
                    if (old == -1 || old == sl) e = k;
                }
                if (e >= 0) atomicAdd(&s_cnt[e], c);
                else atomicSub(&chunks[sl].open, c);  // more chunks than table entries here
            }
            pending &= ~same;
        }
    }
    __syncthreads();
    if (threadIdx.x < kCloseSlots && s_slot[threadIdx.x] >= 0)
        atomicSub(&chunks[s_slot[threadIdx.x]].open, s_cnt[threadIdx.x]);
}

// flag[k] = 1 for clusters (feature rows, ascending label) that are closed
__global__ void k_stream_close_feats(const hc_features* __restrict__ f, const StreamDev* sd, uint64_t dt, int flush,
                                     uint8_t* flag)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= sd->n_all) return;
    const int K = sd->n_clusters;
    const bool hw = sd->has_wmark;
    const uint64_t wmark = sd->wmark;
    flag[k] = (k < K && (flush || (hw && sat_add_u64(f[k].toa_max, dt) <= wmark))) ? 1 : 0;
}

// Stable compaction by flag over the first *n_dev items, in three steps:
// per-block counts, one work-group scan of the counts, scatter.
__global__ __launch_bounds__(kCmpThreads) void k_flag_count(const uint8_t* __restrict__ flag, const int32_t* n_dev,
                                                            uint32_t* counts)
{
    __shared__ uint32_t wsum[kCmpThreads / kWave];
    const int n = *n_dev;
    if ((int64_t)blockIdx.x * kCmpBlock >= n) return;
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

__global__ __launch_bounds__(1024) void k_flag_scan(uint32_t* counts, const int32_t* n_dev, int32_t* total_out)
{
    __shared__ uint32_t wsum[1024 / kWave];
    const int nb = (*n_dev + kCmpBlock - 1) / kCmpBlock;
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

__global__ __launch_bounds__(kCmpThreads) void k_scatter_open(const uint8_t* __restrict__ flag, const int32_t* n_dev,
                                                              const uint32_t* offs, const hc_hit* __restrict__ sb,
                                                              const int32_t* __restrict__ sg,
                                                              const int32_t* __restrict__ sc,
                                                              const int32_t* __restrict__ si, hc_hit* db,
                                                              int32_t* dg, int32_t* dc, int32_t* di)
{
    const int n = *n_dev;
    if ((int64_t)blockIdx.x * kCmpBlock >= n) return;
    flag_scatter(flag, n, offs, [&](int64_t i, uint64_t p) {
        db[p] = sb[i];
        dg[p] = sg[i];
        dc[p] = sc[i];
        if (si) di[p] = si[i];
    });
}

__global__ __launch_bounds__(kCmpThreads) void k_scatter_feats(const uint8_t* __restrict__ flag, const StreamDev* sd,
                                                               const uint32_t* offs,
                                                               const hc_features* __restrict__ f,
                                                               const int32_t* __restrict__ gidx,
                                                               const int32_t* __restrict__ cmin, hc_features* q,
                                                               int64_t q_cap)
{
    const int n = sd->n_all;
    if ((int64_t)blockIdx.x * kCmpBlock >= n) return;
    const int64_t tail = sd->q_tail;
    flag_scatter(flag, n, offs, [&](int64_t k, uint64_t p) {
        hc_features r = f[k];
        r.label = cmin ? cmin[k] : gidx[r.label];  // row k is the cluster of rank k
        q[(tail + (int64_t)p) % q_cap] = r;
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
    uint64_t tag = 0;
    uint64_t reg_seq = 0;  // push that registered the chunk in this slot
    bool active = false;
};

// One enqueued push: its event, and the pinned copy of the device state and
// chunk table taken at its end.
struct PushRec {
    uint64_t seq = 0;
    int slot = -1;          // chunk slot; -1 for a flush
    uint64_t tag = 0;
    int32_t n = 0;
    int mirror_chunks = 0;  // chunk-table entries in the mirror
    hipEvent_t ev = nullptr;
    char* mirror = nullptr;
    size_t mirror_bytes = 0;
};

constexpr int kDefaultDepth = 3;  // pushes in flight at most

}  // namespace

struct hc_stream {
    hipStream_t s = nullptr;   // all pushes
    hipStream_t ds = nullptr;  // copies of closed features to the host (never waits for pushes in flight)
    uint32_t W = 256, H = 256, D = 4096;
    int32_t link_mode = 0;
    uint64_t dt = 0, tdis = 0;
    int depth = kDefaultDepth;
    // open buffer (ping-pong) and per-push scratch, capacity `cap` hits
    int64_t cap = 0;
    int cur = 0;
    hc_hit* buf[2] = {nullptr, nullptr};
    int32_t* gidx[2] = {nullptr, nullptr};
    int32_t* cslot[2] = {nullptr, nullptr};
    int32_t* ids[2] = {nullptr, nullptr};  // caller-supplied ids (streams in id mode)
    int32_t* cmin = nullptr;               // smallest id per cluster of a push
    int id_mode = -1;                      // -1 undecided, 0 global indices, 1 caller ids
    uint8_t* flags = nullptr;
    int32_t* lab = nullptr;
    hc_features* feats = nullptr;
    uint32_t* counts = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // ring of closed-cluster records (device); the host has consumed q_head
    hc_features* queue = nullptr;
    int64_t q_cap = 0, q_head = 0;
    // chunk table
    ChunkRec* chunks_dev = nullptr;
    int chunk_cap = 0;
    std::vector<ChunkHost> chunks;
    std::deque<std::pair<uint64_t, int32_t>> done;  // (tag, status) of finished chunks
    StreamDev* sd = nullptr;
    std::deque<PushRec*> inflight;
    std::vector<PushRec*> spare;
    // known from the pushes completed so far
    int64_t n_open_known = 0, q_tail_known = 0;
    int64_t pushed = 0;        // hits handed to pushes (accepted or not)
    uint64_t seq = 0;          // pushes enqueued
    uint64_t retired = 0;      // pushes completed and read back
    bool failed = false;
    bool log_retired = false;  // keep a record of every completed push (the server reads it)
    std::deque<RetiredPush> retired_log;
};

static void free_rec(PushRec* r)
{
    if (!r) return;
    if (r->ev) (void)hipEventDestroy(r->ev);
    if (r->mirror) (void)hipHostFree(r->mirror);
    delete r;
}

static void free_all(hc_stream* st)
{
    for (int b = 0; b < 2; b++) {
        (void)hipFree(st->buf[b]);
        (void)hipFree(st->gidx[b]);
        (void)hipFree(st->cslot[b]);
        (void)hipFree(st->ids[b]);
    }
    (void)hipFree(st->cmin);
    (void)hipFree(st->flags);
    (void)hipFree(st->lab);
    (void)hipFree(st->feats);
    (void)hipFree(st->counts);
    (void)hipFree(st->ws);
    (void)hipFree(st->queue);
    (void)hipFree(st->chunks_dev);
    (void)hipFree(st->sd);
    for (PushRec* r : st->inflight) free_rec(r);
    for (PushRec* r : st->spare) free_rec(r);
    st->inflight.clear();
    st->spare.clear();
    if (st->ds) (void)hipStreamDestroy(st->ds);
}

// Read back one completed push: rejection, open-hit count, ring tail, and
// the chunks whose labels all became final.
static void retire(hc_stream* st, PushRec* r)
{
    StreamDev d;
    ::memcpy(&d, r->mirror, sizeof(StreamDev));
    const ChunkRec* cr = reinterpret_cast<const ChunkRec*>(r->mirror + sizeof(StreamDev));
    if (d.n_clusters < 0) st->failed = true;
    if (r->slot >= 0 && d.verdict != HC_OK) {
        ChunkHost& c = st->chunks[r->slot];
        st->done.emplace_back(c.tag, d.verdict);
        c.active = false;
    }
    st->n_open_known = d.n_open;
    st->q_tail_known = d.q_tail;
    for (int c = 0; c < r->mirror_chunks; c++) {
        ChunkHost& ch = st->chunks[c];
        if (ch.active && ch.reg_seq <= r->seq && cr[c].open == 0) {
            st->done.emplace_back(ch.tag, HC_OK);
            ch.active = false;
        }
    }
    st->retired = r->seq + 1;
    if (st->log_retired && r->slot >= 0) st->retired_log.push_back(RetiredPush{r->tag, d.verdict, d.n_closed});
}

// Retire completed pushes in order; with `all`, wait for every push.
static int reap(hc_stream* st, bool all)
{
    while (!st->inflight.empty()) {
        PushRec* r = st->inflight.front();
        hipError_t e = hipEventQuery(r->ev);
        if (e == hipErrorNotReady) {
            if (!all) break;
            e = hipEventSynchronize(r->ev);
        }
        if (e != hipSuccess) {
            st->failed = true;
            return set_device_error(e, "stream push");
        }
        retire(st, r);
        st->inflight.pop_front();
        st->spare.push_back(r);
    }
    return HC_OK;
}

static int reap_one(hc_stream* st)
{
    if (st->inflight.empty()) return HC_OK;
    hipError_t e = hipEventSynchronize(st->inflight.front()->ev);
    if (e != hipSuccess) {
        st->failed = true;
        return set_device_error(e, "stream push");
    }
    return reap(st, false);
}

// Upper bound on the open hits once every enqueued push has run: a push
// keeps at most the hits it clusters, i.e. the open ones plus its chunk.
static int64_t open_bound(const hc_stream* st)
{
    int64_t b = st->n_open_known;
    for (const PushRec* r : st->inflight) b += r->n;
    return b;
}

static uint32_t sort_hint(const hc_stream* st)
{
    // the open hits precede the chunk in the buffer; a chunk hit can move up
    // to that many places plus the chunk's own disorder.  A hint only: the
    // last known count of open hits, never the (much larger) bound
    const int64_t h = (int64_t)st->D + st->n_open_known;
    return (uint32_t)(h > 0x7FFFFFFF ? 0x7FFFFFFF : h);
}

// Grow the per-push buffers to hold n_all hits, keeping the open hits
// (waits for the pushes in flight first).
static int ensure_capacity(hc_stream* st, int64_t n_all)
{
    hipError_t e;
    int rc;
    if (n_all > st->cap) {
        if ((rc = reap(st, true)) != HC_OK) return rc;
        int64_t nc = st->cap * 2 > n_all ? st->cap * 2 : n_all;
        if (nc < 4096) nc = 4096;
        hc_hit* nb[2] = {nullptr, nullptr};
        int32_t* ng[2] = {nullptr, nullptr};
        int32_t* ncs[2] = {nullptr, nullptr};
        int32_t* nid[2] = {nullptr, nullptr};
        rc = HC_OK;
        for (int b = 0; b < 2 && rc == HC_OK; b++) {
            if ((rc = dev_alloc(&nb[b], nc)) != HC_OK) break;
            if ((rc = dev_alloc(&ng[b], nc)) != HC_OK) break;
            if ((rc = dev_alloc(&ncs[b], nc)) != HC_OK) break;
            if (st->id_mode == 1) rc = dev_alloc(&nid[b], nc);
        }
        if (rc != HC_OK) {
            for (int b = 0; b < 2; b++) {
                (void)hipFree(nb[b]);
                (void)hipFree(ng[b]);
                (void)hipFree(ncs[b]);
                (void)hipFree(nid[b]);
            }
            return rc;
        }
        const int64_t no = st->n_open_known;
        if (no > 0) {  // the open hits move to the new buffers (all pushes have run)
            e = hipMemcpy(nb[0], st->buf[st->cur], sizeof(hc_hit) * no, hipMemcpyDeviceToDevice);
            if (e == hipSuccess) e = hipMemcpy(ng[0], st->gidx[st->cur], 4 * no, hipMemcpyDeviceToDevice);
            if (e == hipSuccess) e = hipMemcpy(ncs[0], st->cslot[st->cur], 4 * no, hipMemcpyDeviceToDevice);
            if (e == hipSuccess && nid[0] && st->ids[st->cur])
                e = hipMemcpy(nid[0], st->ids[st->cur], 4 * no, hipMemcpyDeviceToDevice);
            if (e != hipSuccess) {
                for (int b = 0; b < 2; b++) {
                    (void)hipFree(nb[b]);
                    (void)hipFree(ng[b]);
                    (void)hipFree(ncs[b]);
                    (void)hipFree(nid[b]);
                }
                st->failed = true;
                return set_device_error(e, "stream buffer growth");
            }
        }
        for (int b = 0; b < 2; b++) {
            (void)hipFree(st->buf[b]);
            (void)hipFree(st->gidx[b]);
            (void)hipFree(st->cslot[b]);
            (void)hipFree(st->ids[b]);
            st->buf[b] = nb[b];
            st->gidx[b] = ng[b];
            st->cslot[b] = ncs[b];
            st->ids[b] = nid[b];
        }
        st->cur = 0;
        (void)hipFree(st->flags);
        (void)hipFree(st->lab);
        (void)hipFree(st->feats);
        (void)hipFree(st->counts);
        (void)hipFree(st->cmin);
        st->flags = nullptr;
        st->lab = nullptr;
        st->feats = nullptr;
        st->counts = nullptr;
        st->cmin = nullptr;
        st->cap = 0;
        if (st->id_mode == 1 && (rc = dev_alloc(&st->cmin, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->flags, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->lab, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->feats, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->counts, (nc + kCmpBlock - 1) / kCmpBlock + 1)) != HC_OK) return rc;
        st->cap = nc;
    }
    const size_t need = plan_workspace(n_all, st->W, st->H, sort_hint(st), nullptr, nullptr);
    if (need > st->ws_bytes) {
        if ((rc = reap(st, true)) != HC_OK) return rc;
        (void)hipFree(st->ws);
        st->ws = nullptr;
        st->ws_bytes = 0;
        const size_t nb = need + need / 4;
        if ((e = hipMalloc(&st->ws, nb)) != hipSuccess) return set_device_error(e, "hipMalloc(stream workspace)");
        st->ws_bytes = nb;
    }
    return HC_OK;
}

// The closed-feature ring must hold every record not yet polled plus what
// the pushes in flight and the next one (n_all hits at most) can close:
// each hit closes once, so at most the open hits plus the chunk hits.
static int ensure_queue(hc_stream* st, int64_t n_all)
{
    const int64_t need = (st->q_tail_known - st->q_head) + n_all;
    if (need <= st->q_cap) return HC_OK;
    int rc = reap(st, true);
    if (rc != HC_OK) return rc;
    const int64_t live = st->q_tail_known - st->q_head;
    int64_t nq = st->q_cap * 2 > live + n_all ? st->q_cap * 2 : live + n_all;
    if (nq < 4096) nq = 4096;
    hc_features* q;
    if ((rc = dev_alloc(&q, nq)) != HC_OK) return rc;
    hipError_t e = hipSuccess;
    if (live > 0) {  // the live records, unwrapped to the front of the new ring
        const int64_t a = st->q_head % st->q_cap;
        const int64_t first = live < st->q_cap - a ? live : st->q_cap - a;
        e = hipMemcpyAsync(q, st->queue + a, sizeof(hc_features) * first, hipMemcpyDeviceToDevice, st->s);
        if (e == hipSuccess && live > first)
            e = hipMemcpyAsync(q + first, st->queue, sizeof(hc_features) * (live - first), hipMemcpyDeviceToDevice,
                               st->s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_stream_set_qtail, dim3(1), dim3(64), 0, st->s, st->sd, (long long)live);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st->s);
    if (e != hipSuccess) {
        (void)hipFree(q);
        return set_device_error(e, "stream ring growth");
    }
    (void)hipFree(st->queue);
    st->queue = q;
    st->q_cap = nq;
    st->q_head = 0;
    st->q_tail_known = live;
    return HC_OK;
}

// Device bytes a stream holds with buffers for `cap` hits, a workspace of
// `ws` bytes, a ring of `q` records and `chunks` chunk slots.
static size_t footprint(int64_t cap, size_t ws, int64_t q, int chunks, bool ids = false)
{
    const size_t per_hit = 2 * (sizeof(hc_hit) + 4 + 4) + 1 + 4 + sizeof(hc_features) + (ids ? 3 * 4 : 0);
    return (size_t)cap * per_hit + 4 * (size_t)((cap + kCmpBlock - 1) / kCmpBlock + 1) + ws +
           sizeof(hc_features) * (size_t)q + sizeof(ChunkRec) * (size_t)chunks + sizeof(StreamDev);
}

static int grow_chunks(hc_stream* st)
{
    hipError_t e;
    int rc = reap(st, true);
    if (rc != HC_OK) return rc;
    const int nc = st->chunk_cap ? st->chunk_cap * 2 : 64;
    ChunkRec* d;
    if ((rc = dev_alloc(&d, nc)) != HC_OK) return rc;
    if (st->chunk_cap &&
        (e = hipMemcpy(d, st->chunks_dev, sizeof(ChunkRec) * st->chunk_cap, hipMemcpyDeviceToDevice)) != hipSuccess) {
        (void)hipFree(d);
        return set_device_error(e, "stream chunk table");
    }
    (void)hipFree(st->chunks_dev);
    st->chunks_dev = d;
    st->chunks.resize(nc);
    st->chunk_cap = nc;
    return HC_OK;
}

static int take_rec(hc_stream* st, PushRec** out)
{
    PushRec* r = nullptr;
    if (!st->spare.empty()) {
        r = st->spare.back();
        st->spare.pop_back();
    } else {
        r = new PushRec();
    }
    hipError_t e = hipSuccess;
    if (!r->ev) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
    const size_t need = sizeof(StreamDev) + sizeof(ChunkRec) * (size_t)st->chunk_cap;
    if (e == hipSuccess && r->mirror_bytes < need) {
        if (r->mirror) (void)hipHostFree(r->mirror);
        r->mirror = nullptr;
        r->mirror_bytes = 0;
        e = hipHostMalloc((void**)&r->mirror, need, hipHostMallocDefault);
        if (e == hipSuccess) r->mirror_bytes = need;
    }
    if (e != hipSuccess) {
        st->spare.push_back(r);
        return set_device_error(e, "stream push record");
    }
    *out = r;
    return HC_OK;
}

// Enqueue one push (or, with flush, the closing of every open cluster):
// append + commit, the plain clustering over the device-resident count,
// closing and compaction, then the pinned read-back of state and chunk table.
static int enqueue_push(hc_stream* st, const hc_hit* hits, const int32_t* in_ids, int32_t n, int slot,
                        int32_t* labels, uint64_t tag, int64_t n_all_bound, int flush)
{
    hipError_t e;
    PushRec* r = nullptr;
    int rc = take_rec(st, &r);
    if (rc != HC_OK) return rc;
    auto give_back = [&](int code) {
        st->spare.push_back(r);
        st->failed = true;  // part of the push may be enqueued: the stream's state is unknown
        return code;
    };
    {
        TimedLaunch tl("stream_append", st->s);
        if (!flush && n > 0)
            hipLaunchKernelGGL(k_stream_append, dim3((n + 255) / 256), dim3(256), 0, st->s, hits, in_ids, n,
                               st->buf[st->cur], st->gidx[st->cur], st->ids[st->cur], st->cslot[st->cur], slot,
                               st->sd, st->tdis, st->W, st->H);
        hipLaunchKernelGGL(k_stream_commit, dim3(1), dim3(64), 0, st->s, st->sd, st->chunks_dev, slot, labels, n,
                           st->tdis, st->dt, flush);
    }
    if ((e = hipGetLastError()) != hipSuccess) return give_back(set_device_error(e, "stream append"));
    const int nxt = 1 - st->cur;
    if (n_all_bound == 0) {
        // a flush with no open hit: nothing to cluster, close or compact
        hipLaunchKernelGGL(k_stream_end, dim3(1), dim3(64), 0, st->s, st->sd);
        if ((e = hipGetLastError()) != hipSuccess) return give_back(set_device_error(e, "stream close"));
    } else {
        Work w;
        plan_workspace(n_all_bound, st->W, st->H, sort_hint(st), &w, (char*)st->ws);
        w.dt = st->dt;
        w.link_mode = st->link_mode;
        w.n_dev = &st->sd->n_all;
        if ((rc = enqueue_cluster(st->buf[st->cur], w, st->lab, st->feats, &st->sd->n_clusters, st->s)) != HC_OK)
            return give_back(rc);
        const int nb_all = (int)((n_all_bound + 255) / 256);
        const int nb = (int)((n_all_bound + kCmpBlock - 1) / kCmpBlock);
        {
            TimedLaunch tl("stream_close", st->s);  // the closing and compaction kernels, together
            const int32_t* cmin = st->id_mode == 1 ? st->cmin : nullptr;
            if (cmin) {
                hipLaunchKernelGGL(k_stream_idmin_init, dim3(nb_all), dim3(256), 0, st->s, st->cmin, st->sd);
                hipLaunchKernelGGL(k_stream_idmin, dim3(nb_all), dim3(256), 0, st->s, st->lab, w, st->ids[st->cur],
                                   st->sd, st->cmin);
            }
            hipLaunchKernelGGL(k_stream_close_hits, dim3((int)((n_all_bound + kCloseBlock - 1) / kCloseBlock)),
                               dim3(kCloseThreads), 0, st->s, st->lab, w, st->gidx[st->cur], st->cslot[st->cur], cmin,
                               st->chunks_dev, st->sd, st->dt, flush, st->flags);
            hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, &st->sd->n_all, st->counts);
            hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st->s, st->counts, &st->sd->n_all, &st->sd->n_open);
            hipLaunchKernelGGL(k_scatter_open, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, &st->sd->n_all,
                               st->counts, st->buf[st->cur], st->gidx[st->cur], st->cslot[st->cur], st->ids[st->cur],
                               st->buf[nxt], st->gidx[nxt], st->cslot[nxt], st->ids[nxt]);
            hipLaunchKernelGGL(k_stream_close_feats, dim3(nb_all), dim3(256), 0, st->s, st->feats, st->sd, st->dt, flush,
                               st->flags);
            hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, &st->sd->n_all, st->counts);
            hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st->s, st->counts, &st->sd->n_all, &st->sd->n_closed);
            hipLaunchKernelGGL(k_scatter_feats, dim3(nb), dim3(kCmpThreads), 0, st->s, st->flags, st->sd, st->counts,
                               st->feats, st->gidx[st->cur], cmin, st->queue, st->q_cap);
            hipLaunchKernelGGL(k_stream_end, dim3(1), dim3(64), 0, st->s, st->sd);
        }
        if ((e = hipGetLastError()) != hipSuccess) return give_back(set_device_error(e, "stream close"));
    }
    if ((e = hipMemcpyAsync(r->mirror, st->sd, sizeof(StreamDev), hipMemcpyDeviceToHost, st->s)) != hipSuccess ||
        (e = hipMemcpyAsync(r->mirror + sizeof(StreamDev), st->chunks_dev, sizeof(ChunkRec) * st->chunk_cap,
                            hipMemcpyDeviceToHost, st->s)) != hipSuccess ||
        (e = hipEventRecord(r->ev, st->s)) != hipSuccess)
        return give_back(set_device_error(e, "stream read-back"));
    r->seq = st->seq++;
    r->slot = slot;
    r->tag = tag;
    r->n = flush ? 0 : n;
    r->mirror_chunks = st->chunk_cap;
    st->inflight.push_back(r);
    if (slot >= 0) {
        st->chunks[slot].tag = tag;
        st->chunks[slot].reg_seq = r->seq;
        st->chunks[slot].active = true;
    }
    st->cur = nxt;
    return HC_OK;
}

namespace hc {

size_t stream_device_bytes(const hc_stream* st)
{
    return footprint(st->cap, st->ws_bytes, st->q_cap, st->chunk_cap, st->id_mode == 1);
}

// What the stream may hold after enqueuing a push of n hits (the growth
// rules of ensure_capacity, ensure_queue and grow_chunks); *transient: bytes
// of old buffers alive together with their replacements while growing.
size_t stream_bytes_after_push(const hc_stream* st, int64_t n, size_t* transient)
{
    const int64_t n_all = open_bound(st) + n;
    int64_t cap = st->cap;
    size_t tr = 0;
    if (n_all > cap) {
        cap = st->cap * 2 > n_all ? st->cap * 2 : n_all;
        if (cap < 4096) cap = 4096;
        tr += footprint(st->cap, 0, 0, 0);
    }
    const size_t need = plan_workspace(n_all, st->W, st->H, sort_hint(st), nullptr, nullptr);
    const size_t ws = need > st->ws_bytes ? need + need / 4 : st->ws_bytes;
    int64_t q = st->q_cap;
    const int64_t qneed = (st->q_tail_known - st->q_head) + n_all;
    if (qneed > q) {
        q = st->q_cap * 2 > qneed ? st->q_cap * 2 : qneed;
        if (q < 4096) q = 4096;
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
    return footprint(cap, ws, q, chunks, st->id_mode == 1);
}

int64_t stream_open_hits(const hc_stream* st) { return st->n_open_known; }

uint64_t stream_pushes_retired(hc_stream* st)
{
    (void)reap(st, false);
    return st->retired;
}

uint64_t stream_pushes_enqueued(const hc_stream* st) { return st->seq; }

int stream_wait_one(hc_stream* st) { return reap_one(st); }

void stream_configure(hc_stream* st, int depth, bool log_retired)
{
    st->depth = depth < 1 ? 1 : depth;
    st->log_retired = log_retired;
}

size_t stream_take_retired(hc_stream* st, std::vector<RetiredPush>* out)
{
    (void)reap(st, false);
    const size_t k = st->retired_log.size();
    out->insert(out->end(), st->retired_log.begin(), st->retired_log.end());
    st->retired_log.clear();
    return k;
}

size_t stream_inflight(const hc_stream* st) { return st->inflight.size(); }

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
    if (st->W > 65535 || st->H > 65535 || (opts && !link_flags_valid(opts->flags)) || global_time_of(opts)) {
        delete st;
        return set_error(HC_ERR_ARG, "bad stream options");
    }
    hipError_t e;
    int rc = dev_alloc(&st->sd, 1);
    if (rc == HC_OK && (e = hipMemsetAsync(st->sd, 0, sizeof(StreamDev), st->s)) != hipSuccess)
        rc = set_device_error(e, "stream state");
    if (rc == HC_OK && (e = hipStreamCreateWithFlags(&st->ds, hipStreamNonBlocking)) != hipSuccess)
        rc = set_device_error(e, "hipStreamCreate");
    if (rc == HC_OK) rc = grow_chunks(st);
    if (rc == HC_OK && (e = hipStreamSynchronize(st->s)) != hipSuccess) rc = set_device_error(e, "stream create");
    if (rc != HC_OK) {
        free_all(st);
        delete st;
        return rc;
    }
    *out = st;
    return HC_OK;
}

// First push of a stream with caller ids: give the per-hit buffers their id
// arrays (nothing is open yet, so nothing has to be carried over).
static int enter_id_mode(hc_stream* st)
{
    int rc = reap(st, true);
    if (rc != HC_OK) return rc;
    st->id_mode = 1;
    if (st->cap > 0) {
        for (int b = 0; b < 2 && rc == HC_OK; b++) rc = dev_alloc(&st->ids[b], st->cap);
        if (rc == HC_OK) rc = dev_alloc(&st->cmin, st->cap);
    }
    return rc;
}

static int push_impl(hc_stream* st, const hc_hit* hits, const int32_t* ids, int32_t n, int32_t* labels,
                     uint64_t tag)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    if (n < 0 || (n > 0 && (!hits || !labels || (st->id_mode == 1 && !ids))))
        return set_error(HC_ERR_ARG, "bad chunk arguments");
    const int mode = ids ? 1 : 0;
    if (n > 0 && st->id_mode >= 0 && st->id_mode != mode)
        return set_error(HC_ERR_ARG, "a stream takes ids with every push or with none");
    if (st->pushed + n > 0x7FFFFFFF) return set_error(HC_ERR_OVERFLOW, "more than 2^31 - 1 hits in the stream");
    if (n == 0) {
        st->done.emplace_back(tag, HC_OK);
        return HC_OK;
    }
    int rc = HC_OK;
    if (st->id_mode < 0) {
        if (mode == 1) {
            if ((rc = enter_id_mode(st)) != HC_OK) return rc;
        } else {
            st->id_mode = 0;
        }
    }
    rc = reap(st, false);
    while (rc == HC_OK && (int)st->inflight.size() >= st->depth) rc = reap_one(st);
    if (rc != HC_OK) return rc;
    int slot = -1;
    for (int c = 0; c < st->chunk_cap && slot < 0; c++)
        if (!st->chunks[c].active) slot = c;
    if (slot < 0) {
        if ((rc = grow_chunks(st)) != HC_OK) return rc;
        for (int c = 0; c < st->chunk_cap && slot < 0; c++)
            if (!st->chunks[c].active) slot = c;
    }
    if ((rc = ensure_capacity(st, open_bound(st) + n)) != HC_OK) return rc;
    if ((rc = ensure_queue(st, open_bound(st) + n)) != HC_OK) return rc;
    // a growth above may have waited for the pushes in flight, which tightens
    // the bound and changes the sort hint: size the workspace for the final plan
    const int64_t n_all = open_bound(st) + n;
    if ((rc = ensure_capacity(st, n_all)) != HC_OK) return rc;
    if ((rc = enqueue_push(st, hits, ids, n, slot, labels, tag, n_all, 0)) != HC_OK) return rc;
    st->pushed += n;
    return HC_OK;
}

int hc_stream_push(hc_stream* st, const hc_hit* hits, int32_t n, int32_t* labels, uint64_t tag)
{
    return push_impl(st, hits, nullptr, n, labels, tag);
}

int hc_stream_push_ids(hc_stream* st, const hc_hit* hits, const int32_t* ids, int32_t n, int32_t* labels,
                       uint64_t tag)
{
    if (n > 0 && !ids) return set_error(HC_ERR_ARG, "ids is NULL");
    return push_impl(st, hits, ids, n, labels, tag);
}

int hc_stream_reserve(hc_stream* st, int32_t max_chunk)
{
    if (!st || max_chunk < 0) return set_error(HC_ERR_ARG, "bad stream or size");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    int rc = reap(st, true);
    if (rc != HC_OK) return rc;
    // open hits carried between pushes, plus a full set of pushes in flight
    const int64_t margin = max_chunk / 4 + 4096;
    const int64_t open = st->n_open_known > margin ? st->n_open_known : margin;
    const int64_t n_all = open + (int64_t)st->depth * max_chunk;
    // the workspace for the sort hint of `open` open hits
    const int64_t keep = st->n_open_known;
    st->n_open_known = open;
    const size_t need = plan_workspace(n_all, st->W, st->H, sort_hint(st), nullptr, nullptr);
    st->n_open_known = keep;
    if ((rc = ensure_capacity(st, n_all)) != HC_OK) return rc;
    if (need > st->ws_bytes) {
        hipError_t e;
        (void)hipFree(st->ws);
        st->ws = nullptr;
        st->ws_bytes = 0;
        if ((e = hipMalloc(&st->ws, need)) != hipSuccess) return set_device_error(e, "hipMalloc(stream workspace)");
        st->ws_bytes = need;
    }
    return ensure_queue(st, n_all);
}

int64_t hc_stream_open_hits(const hc_stream* st) { return st ? st->n_open_known : -1; }

int hc_stream_wait(hc_stream* st)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    int rc = reap(st, true);
    if (rc != HC_OK) return rc;
    return st->failed ? set_error(HC_ERR_DEVICE, "stream: internal clustering error") : HC_OK;
}

int hc_stream_flush(hc_stream* st)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    int rc = reap(st, false);
    if (rc != HC_OK) return rc;
    if ((rc = ensure_capacity(st, open_bound(st))) != HC_OK) return rc;
    if ((rc = ensure_queue(st, open_bound(st))) != HC_OK) return rc;
    const int64_t n_all = open_bound(st);
    if ((rc = ensure_capacity(st, n_all)) != HC_OK) return rc;
    if ((rc = enqueue_push(st, nullptr, nullptr, 0, -1, nullptr, 0, n_all, 1)) != HC_OK) return rc;
    return hc_stream_wait(st);
}

int hc_stream_poll(hc_stream* st, uint64_t* done_tags, int32_t* status, int32_t cap, int32_t* n_done,
                   hc_features* closed, int32_t closed_cap, int32_t* n_closed)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    int rc = reap(st, false);
    if (rc != HC_OK) return rc;
    int32_t nd = 0;
    while (nd < cap && !st->done.empty() && done_tags) {
        done_tags[nd] = st->done.front().first;
        if (status) status[nd] = st->done.front().second;
        nd++;
        st->done.pop_front();
    }
    if (n_done) *n_done = nd;
    int32_t nc = 0;
    const int64_t avail = st->q_tail_known - st->q_head;
    if (closed && closed_cap > 0 && avail > 0) {
        nc = (int32_t)(avail < closed_cap ? avail : closed_cap);
        // records below the tail of a completed push are complete; the copy
        // runs on the drain stream, so it never waits for pushes in flight
        const int64_t a = st->q_head % st->q_cap;
        const int64_t first = nc < st->q_cap - a ? nc : st->q_cap - a;
        hipError_t e =
            hipMemcpyAsync(closed, st->queue + a, sizeof(hc_features) * first, hipMemcpyDeviceToHost, st->ds);
        if (e == hipSuccess && nc > first)
            e = hipMemcpyAsync(closed + first, st->queue, sizeof(hc_features) * (nc - first), hipMemcpyDeviceToHost,
                               st->ds);
        if (e == hipSuccess) e = hipStreamSynchronize(st->ds);
        if (e != hipSuccess) return set_device_error(e, "stream poll");
        st->q_head += nc;
    }
    if (n_closed) *n_closed = nc;
    return st->failed ? set_error(HC_ERR_DEVICE, "stream: internal clustering error") : HC_OK;
}

void hc_stream_destroy(hc_stream* st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->s);
    if (st->ds) (void)hipStreamSynchronize(st->ds);
    free_all(st);
    delete st;
}

}  // extern "C"
