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
// index, M, the closed-feature ring's tail) lives in device memory, the last
// work-group of the append kernel accepts or rejects each chunk on the
// device, and the clustering kernels read their hit count from there (the
// host sizes the grids with an upper bound).  The closing is two kernels: one
// pass decides every hit and cluster and counts per work-group (the last
// work-group turns the counts into offsets), one pass moves the open hits and
// the closed clusters' records.  After each push one pinned copy of the state
// and the chunk table is taken; the host reads it once the push's event
// completes.
#include <string.h>

#include <deque>
#include <string>
#include <vector>

#include "hc_device.h"

namespace hc {

// A push carries one chunk, or several chunks of the stream back to back
// (kMaxPushChunks at most), each accepted or rejected on its own exactly as
// if it had been pushed alone, in order.

// The chunks of one push (a kernel argument): chunk j is hits
// [start[j], start[j + 1]) of the push's input, registered in chunk slot
// slot[j] with the caller's label buffer labels[j].
struct PushChunks {
    int32_t k;
    int32_t start[kMaxPushChunks + 1];
    int32_t slot[kMaxPushChunks];
    int32_t* labels[kMaxPushChunks];
};

// chunk flags raised by its hits
constexpr int32_t kOffSensor = 1, kBadId = 2, kLate = 4;

struct StreamDev {
    // across pushes
    int32_t n_open;               // open hits at the front of the current buffer
    int32_t next_g;               // global index of the next accepted hit
    unsigned long long M;         // largest accepted ToA (valid when has_M)
    unsigned long long floor;     // after a flush, later hits need toa > floor
    int32_t has_M, has_floor;
    long long q_tail;             // closed-feature records written so far (ring slot q_tail % q_cap)
    // the current push
    int32_t n_all;                // hits the push clusters: the open ones, plus its accepted chunks
    int32_t n_closed;             // clusters closed by the push
    int32_t n_clusters;           // clusters of the buffer (or an error status)
    int32_t has_wmark;
    unsigned long long wmark;     // closing watermark of the push (valid when has_wmark)
    uint32_t ticket;              // work-groups of the running kernel done so far (last one resets it)
    // per chunk of the push: ~(smallest ToA) and largest ToA (0 when unset),
    // flags; then, from the commit, its buffer position (-1: rejected) and the
    // global index of its first hit
    unsigned long long c_inv_min[kMaxPushChunks], c_max[kMaxPushChunks];
    int32_t c_flags[kMaxPushChunks], c_dest[kMaxPushChunks], c_base[kMaxPushChunks];
    long long q_base;             // q_tail before the push's closed records (set by the closing)
};

// The stream state and the chunk table share one device block (state at
// offset 0, table at kStateHdr), read back by one copy after every push.
constexpr size_t kStateHdr = 1024;
static_assert(sizeof(StreamDev) <= kStateHdr, "state header");

// Whether this work-group is the last of `active` to get here.  What a
// work-group hands to the last one it writes from its first wave (after
// reducing it in the group), so one fence per group suffices: every such write is visible
// to the work-group that gets true, which also resets the ticket for the next
// kernel.  No work-group waits for another.
__device__ inline bool last_group(StreamDev* sd, uint32_t active)
{
    __shared__ int s_last;
    __syncthreads();  // every wave of the group is past its work
    if (threadIdx.x < kWave) __threadfence();  // the first wave's writes (the group's results)
    if (threadIdx.x == 0) {
        s_last = atomicAdd(&sd->ticket, 1u) == active - 1;
        if (s_last) sd->ticket = 0;
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last;
}

struct ChunkRec {
    int32_t* labels;  // caller's buffer for the chunk's labels
    int64_t base;     // global index of the chunk's first hit (-1: rejected)
    int32_t count;
    int32_t open;     // hits whose label is not final yet
    int32_t verdict;  // HC_OK, or why the chunk was rejected
    int32_t unused_;
};

constexpr int kCmpBlock = 2048;
constexpr int kCmpThreads = 256;
// per-block count entries for `cap` hits (one array each for hits and rows)
constexpr int64_t count_slots(int64_t cap) { return (cap + kCmpBlock - 1) / kCmpBlock + 1; }

__device__ inline uint64_t sat_add_u64(uint64_t a, uint64_t b) { return ~0ull - a < b ? ~0ull : a + b; }

__device__ void commit_chunks(StreamDev* sd, ChunkRec* chunks, const PushChunks& pc, uint64_t tdis);

// The ToA threshold of the stream's contract: later hits need toa > thr
// (has_thr), from the watermark M - t once M >= t and the floor after a flush.
__device__ inline bool contract_threshold(const StreamDev& d, uint64_t tdis, uint64_t* thr)
{
    const bool has_w = d.has_M && d.M >= tdis;
    uint64_t t = has_w ? d.M - tdis : 0;
    bool has = has_w;
    if (d.has_floor) {
        if (!has || d.floor > t) t = d.floor;
        has = true;
    }
    *thr = t;
    return has;
}

// A push of one chunk: copy it behind the open hits and check it against the
// stream's contract (every hit on the sensor, and above the threshold).  A
// work-group takes kAppendBlock hits; the last one to finish commits the
// chunk.
constexpr int kAppendBlock = 2048;

__global__ __launch_bounds__(256) void k_stream_append(const hc_hit* __restrict__ in,
                                                       const int32_t* __restrict__ in_ids, const PushChunks pc,
                                                       hc_hit* buf, int32_t* gidx, int32_t* ids, int32_t* cslot,
                                                       StreamDev* sd, ChunkRec* chunks, uint64_t tdis, uint32_t W,
                                                       uint32_t H)
{
    __shared__ uint64_t red[256 / kWave];
    const int n = pc.start[1];
    const int slot = pc.slot[0];
    const int n_open = sd->n_open;
    const int32_t base = sd->next_g;
    uint64_t thr;
    const bool has_thr = contract_threshold(*sd, tdis, &thr);
    uint64_t mx = 0;
    bool bad_id = false, late = false, off = false;
    for (int q = 0; q < kAppendBlock / 256; q++) {
        const int i = blockIdx.x * kAppendBlock + q * 256 + threadIdx.x;
        if (i >= n) break;
        const hc_hit h = in[i];
        buf[n_open + i] = h;
        gidx[n_open + i] = base + i;
        cslot[n_open + i] = slot;
        if (ids) {
            const int32_t id = in_ids ? in_ids[i] : base + i;
            ids[n_open + i] = id;
            bad_id |= id < 0;
        }
        mx = h.toa > mx ? h.toa : mx;
        late |= has_thr && h.toa <= thr;
        off |= h.x >= W || h.y >= H;
    }
    mx = block_max_u64<256>(mx, red);
    bad_id = __syncthreads_or(bad_id);
    late = __syncthreads_or(late);
    off = __syncthreads_or(off);
    if (threadIdx.x == 0) {  // the group's results, from its first wave (see last_group)
        atomicMax(&sd->c_max[0], (unsigned long long)mx);
        const int32_t f = (off ? kOffSensor : 0) | (bad_id ? kBadId : 0) | (late ? kLate : 0);
        if (f) atomicOr(&sd->c_flags[0], f);
    }
    if (last_group(sd, gridDim.x) && threadIdx.x == 0) commit_chunks(sd, chunks, pc, tdis);
}

// The chunks of a push in LDS, and the chunk of input hit i.
__device__ inline void load_chunks(const PushChunks& pc, int32_t* s_start, int32_t* s_slot)
{
    if (threadIdx.x <= (unsigned)pc.k) s_start[threadIdx.x] = pc.start[threadIdx.x];
    if (threadIdx.x < (unsigned)pc.k) s_slot[threadIdx.x] = pc.slot[threadIdx.x];
    __syncthreads();
}

__device__ inline int chunk_of(const int32_t* s_start, int k, int i)
{
    int j = 0;
    while (j + 1 < k && i >= s_start[j + 1]) j++;
    return j;
}

// A push of several chunks, first pass: each chunk's smallest and largest ToA
// and flags (its acceptance depends on the chunks before it, so the contract
// is checked by the commit, which the last work-group runs).
__global__ __launch_bounds__(256) void k_stream_chunk_stats(const hc_hit* __restrict__ in,
                                                            const int32_t* __restrict__ in_ids, const PushChunks pc,
                                                            StreamDev* sd, ChunkRec* chunks, int ids_mode,
                                                            uint64_t tdis, uint32_t W, uint32_t H)
{
    __shared__ int32_t s_start[kMaxPushChunks + 1], s_slot[kMaxPushChunks];
    __shared__ unsigned long long s_inv_min[kMaxPushChunks], s_max[kMaxPushChunks];
    __shared__ int32_t s_flags[kMaxPushChunks];
    if (threadIdx.x < kMaxPushChunks) {
        s_inv_min[threadIdx.x] = 0;
        s_max[threadIdx.x] = 0;
        s_flags[threadIdx.x] = 0;
    }
    load_chunks(pc, s_start, s_slot);
    const int n = s_start[pc.k];
    for (int q = 0; q < kAppendBlock / 256; q++) {
        const int i = blockIdx.x * kAppendBlock + q * 256 + threadIdx.x;
        if (i >= n) break;
        const int j = chunk_of(s_start, pc.k, i);
        const hc_hit h = in[i];
        atomicMax(&s_inv_min[j], ~(unsigned long long)h.toa);
        atomicMax(&s_max[j], (unsigned long long)h.toa);
        const int32_t f = ((h.x >= W || h.y >= H) ? kOffSensor : 0) | ((ids_mode && in_ids && in_ids[i] < 0) ? kBadId : 0);
        if (f) atomicOr(&s_flags[j], f);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)pc.k) {  // first wave (k <= kMaxPushChunks < kWave)
        const int j = threadIdx.x;
        if (s_max[j] || s_inv_min[j]) {
            atomicMax(&sd->c_inv_min[j], s_inv_min[j]);
            atomicMax(&sd->c_max[j], s_max[j]);
        }
        if (s_flags[j]) atomicOr(&sd->c_flags[j], s_flags[j]);
    }
    if (last_group(sd, gridDim.x) && threadIdx.x == 0) commit_chunks(sd, chunks, pc, tdis);
}

// Second pass: the hits of every accepted chunk behind the open hits and the
// accepted chunks before it.
__global__ __launch_bounds__(256) void k_stream_place(const hc_hit* __restrict__ in, const int32_t* __restrict__ in_ids,
                                                      const PushChunks pc, const StreamDev* sd, hc_hit* buf,
                                                      int32_t* gidx, int32_t* ids, int32_t* cslot)
{
    __shared__ int32_t s_start[kMaxPushChunks + 1], s_slot[kMaxPushChunks];
    __shared__ int32_t s_dest[kMaxPushChunks], s_base[kMaxPushChunks];
    if (threadIdx.x < (unsigned)pc.k) {
        s_dest[threadIdx.x] = sd->c_dest[threadIdx.x];
        s_base[threadIdx.x] = sd->c_base[threadIdx.x];
    }
    load_chunks(pc, s_start, s_slot);
    const int n = s_start[pc.k];
    for (int q = 0; q < kAppendBlock / 256; q++) {
        const int i = blockIdx.x * kAppendBlock + q * 256 + threadIdx.x;
        if (i >= n) break;
        const int j = chunk_of(s_start, pc.k, i);
        if (s_dest[j] < 0) continue;
        const int off = i - s_start[j];
        const int p = s_dest[j] + off;
        buf[p] = in[i];
        gidx[p] = s_base[j] + off;
        cslot[p] = s_slot[j];
        if (ids) ids[p] = in_ids ? in_ids[i] : s_base[j] + off;
    }
}

// Accept or reject the chunks of a push in order (one thread), each as if it
// had been pushed alone: an accepted chunk is registered in the chunk table,
// gets the next global indices and buffer positions, and M advances (which
// raises the threshold for the chunks after it); a rejected one is left out
// (its hits are not clustered) and closes nothing.  The closing watermark
// follows the final M.
__device__ void commit_chunks(StreamDev* sd, ChunkRec* chunks, const PushChunks& pc, uint64_t tdis)
{
    StreamDev& d = *sd;
    d.n_closed = 0;
    d.n_clusters = 0;  // set by the clustering, which a push with nothing to cluster skips
    int32_t n_all = d.n_open;
    uint64_t thr;
    bool has_thr = contract_threshold(d, tdis, &thr);
    for (int j = 0; j < pc.k; j++) {
        const int32_t cnt = pc.start[j + 1] - pc.start[j];
        const int32_t f = d.c_flags[j];
        const bool late = (f & kLate) || (has_thr && ~d.c_inv_min[j] <= thr);
        const int32_t v = (f & kBadId) ? HC_ERR_ARG : (f & kOffSensor) ? HC_ERR_RANGE : late ? HC_ERR_DISORDER : HC_OK;
        if (v == HC_OK) {
            chunks[pc.slot[j]] = ChunkRec{pc.labels[j], (int64_t)d.next_g, cnt, cnt, HC_OK, 0};
            d.c_dest[j] = n_all;
            d.c_base[j] = d.next_g;
            n_all += cnt;
            d.next_g += cnt;
            const unsigned long long mx = d.c_max[j];
            d.M = d.has_M ? (mx > d.M ? mx : d.M) : mx;
            d.has_M = 1;
            has_thr = contract_threshold(d, tdis, &thr);
        } else {
            chunks[pc.slot[j]] = ChunkRec{pc.labels[j], -1, cnt, 0, v, 0};
            d.c_dest[j] = -1;
        }
        d.c_inv_min[j] = 0;  // neutral for the next push
        d.c_max[j] = 0;
        d.c_flags[j] = 0;
    }
    d.n_all = n_all;
    d.has_wmark = d.has_M && d.M >= tdis;
    d.wmark = d.has_wmark ? d.M - tdis : 0;
}

// A flush (one thread): nothing is appended; the open hits are clustered and
// all of them closed, and the floor M + dt applies to whatever comes later.
__global__ void k_stream_commit_flush(StreamDev* sd, uint64_t dt)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    StreamDev& d = *sd;
    d.n_closed = 0;
    d.n_clusters = 0;
    d.n_all = d.n_open;
    d.has_wmark = 0;
    d.wmark = 0;
    if (d.has_M) {
        d.floor = sat_add_u64(d.M, dt);
        d.has_floor = 1;
    }
}

// End of a push: advance the ring's tail.
__device__ inline void end_push(StreamDev* sd) { sd->q_tail += sd->n_closed; }

__global__ void k_stream_end(StreamDev* sd)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) end_push(sd);
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

// The closing of a push, one pass over the clustered hits and the feature
// rows (both in blocks of kCloseBlock).  A hit is final when its cluster is
// closed: its stream-global label goes into its chunk's buffer, and keep[i] =
// 1 for the hits that stay open; fflag[k] = 1 for the closed clusters
// (feature rows, ascending label).  Every chunk counts its hits whose labels
// are not final yet; the decrements go through a small per-work-group table
// in LDS (a work-group's hits mostly come from one or two chunks), one global
// atomic per chunk and work-group, since atomics on one address from every
// wave serialise in the L2.  Each work-group counts its kept hits and closed
// rows; the last one to finish turns both count arrays into exclusive
// offsets for the stable compactions and writes the totals.
constexpr int kCloseThreads = 256;
constexpr int kCloseBlock = 2048;
constexpr int kCloseSlots = 8;
static_assert(kCloseBlock == kCmpBlock, "closing and compaction share their blocks");

__device__ inline void scan_counts_in_place(uint32_t* c, int nb, int32_t* total_out, uint32_t* wsum)
{
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kCloseThreads) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < nb ? c[i] : 0u;
        uint32_t total;
        const uint32_t e = block_exclusive_scan<kCloseThreads>(v, wsum, &total);
        if (i < nb) c[i] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = (int32_t)carry;
}

__global__ __launch_bounds__(kCloseThreads) void k_stream_close(const int32_t* __restrict__ lab, const Work w,
                                                                const int32_t* __restrict__ gidx,
                                                                const int32_t* __restrict__ cslot,
                                                                const int32_t* __restrict__ cmin,
                                                                const hc_features* __restrict__ f,
                                                                ChunkRec* chunks, StreamDev* sd, uint64_t dt,
                                                                int flush, uint8_t* keep, uint8_t* fflag,
                                                                uint32_t* hcount, uint32_t* fcount)
{
    __shared__ int32_t s_slot[kCloseSlots];
    __shared__ int32_t s_cnt[kCloseSlots];
    __shared__ uint32_t wsum[kCloseThreads / kWave];
    const int n_all = sd->n_all;
    if (sd->n_clusters < 0) return;  // the clustering failed; the host reports it
    if (n_all == 0) {                // nothing clustered: nothing stays open or closes
        if (blockIdx.x == 0 && threadIdx.x == 0) sd->n_open = 0;
        return;
    }
    const int nb = (n_all + kCloseBlock - 1) / kCloseBlock;
    if ((int)blockIdx.x >= nb) return;
    if (threadIdx.x < kCloseSlots) {
        s_slot[threadIdx.x] = -1;
        s_cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    const int K = sd->n_clusters;
    const bool has_wmark = sd->has_wmark;
    const uint64_t wmark = sd->wmark;
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int Q = kCloseBlock / kCloseThreads;
    // each level's loads for all Q hits of the thread go out together (label,
    // then the root's rank, then the cluster's last ToA), so a thread waits
    // for three round trips rather than three per hit
    int32_t r[Q], cs[Q], gi[Q];
    uint64_t fmax[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int64_t i = (int64_t)blockIdx.x * kCloseBlock + q * kCloseThreads + threadIdx.x;
        const bool in = i < n_all;
        r[q] = in ? lab[i] : 0;
        cs[q] = in ? cslot[i] : 0;
        gi[q] = in ? gidx[i] : 0;
        fmax[q] = (in && i < K) ? f[i].toa_max : 0;
    }
    uint32_t rank[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int64_t i = (int64_t)blockIdx.x * kCloseBlock + q * kCloseThreads + threadIdx.x;
        if (i < n_all && (r[q] < 0 || r[q] > i)) {
            atomicOr(&w.status->err_internal, 1);
            r[q] = (int32_t)i;
        }
        rank[q] = i < n_all ? root_rank(w, 0, 0, r[q]) : 0u;
    }
    uint64_t tmax[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int64_t i = (int64_t)blockIdx.x * kCloseBlock + q * kCloseThreads + threadIdx.x;
        tmax[q] = i < n_all ? w.slots[rank[q]].toa_max : 0;
    }
    uint32_t kept = 0, fclosed = 0;
    for (int q = 0; q < Q; q++) {
        const int64_t i = (int64_t)blockIdx.x * kCloseBlock + q * kCloseThreads + threadIdx.x;
        bool closed = false;
        int32_t slot = -1;
        if (i < n_all) {
            closed = flush || (has_wmark && sat_add_u64(tmax[q], dt) <= wmark);
            if (closed) {
                slot = cs[q];
                ChunkRec* ch = chunks + slot;
                ch->labels[gi[q] - ch->base] = cmin ? cmin[rank[q]] : gidx[r[q]];
            }
            keep[i] = closed ? 0 : 1;
            kept += closed ? 0u : 1u;
            // feature row i (rows beyond the clusters are never closed)
            const bool fc = i < K && (flush || (has_wmark && sat_add_u64(fmax[q], dt) <= wmark));
            fflag[i] = fc ? 1 : 0;
            fclosed += fc ? 1u : 0u;
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
    uint32_t kt, ft;
    (void)block_exclusive_scan<kCloseThreads>(kept, wsum, &kt);
    (void)block_exclusive_scan<kCloseThreads>(fclosed, wsum, &ft);
    if (threadIdx.x == 0) {
        hcount[blockIdx.x] = kt;
        fcount[blockIdx.x] = ft;
    }
    if (threadIdx.x < kCloseSlots && s_slot[threadIdx.x] >= 0)
        atomicSub(&chunks[s_slot[threadIdx.x]].open, s_cnt[threadIdx.x]);
    if (!last_group(sd, (uint32_t)nb)) return;
    scan_counts_in_place(hcount, nb, &sd->n_open, wsum);
    scan_counts_in_place(fcount, nb, &sd->n_closed, wsum);
    if (threadIdx.x == 0) sd->q_base = sd->q_tail;
}

// Stable compaction of block b's flagged items, emitting those of slices
// [q0, q1).  Lanes take consecutive items (slice q holds items
// b * kCmpBlock + q * kCmpThreads + t), so reads and writes of runs of
// flagged items coalesce; an item's place is off (the block's first) plus the
// flagged items of earlier slices, of earlier waves in its slice and of
// earlier lanes in its wave.
template <class F>
__device__ inline void flag_scatter(const uint8_t* __restrict__ flag, int n, int b, uint32_t off, int q0, int q1,
                                    F&& emit)
{
    constexpr int PER = kCmpBlock / kCmpThreads;
    constexpr int NW = kCmpThreads / kWave;
    __shared__ uint32_t wcnt[PER * NW];
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
    const int64_t b0 = (int64_t)b * kCmpBlock;
    unsigned long long bal[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t i = b0 + q * kCmpThreads + t;
        bal[q] = __ballot(i < n && flag[i] != 0);
        if (lane == 0) wcnt[q * NW + wv] = (uint32_t)__popcll(bal[q]);
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t pos = off;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < NW; k++) {
            const uint32_t c = wcnt[q * NW + k];
            before += k < wv ? c : 0u;
            all += c;
        }
        if (q >= q0 && q < q1 && ((bal[q] >> lane) & 1ull))
            emit(b0 + q * kCmpThreads + t, (uint64_t)pos + before + (uint32_t)__popcll(bal[q] & below));
        pos += all;
    }
    __syncthreads();  // wcnt is read before another call writes it
}

// Both stable compactions of a push: the open hits to the front of the other
// buffer, the closed clusters' features (with their stream-global labels) to
// the ring.  Work-groups [0, nb_grid) take one block of hits each, and the
// last of them to finish ends the push; the next nb_grid * PER take one slice
// of kCmpThreads feature rows each (only the first rows of a push are feature
// rows, so blocks of rows would leave most work-groups idle).  The rows go
// behind q_base, which the closing set, so they never read the tail that the
// end of the push moves.
__global__ __launch_bounds__(kCmpThreads) void k_stream_scatter(
    const uint8_t* __restrict__ keep, const uint8_t* __restrict__ fflag, const uint32_t* hoff, const uint32_t* foff,
    StreamDev* sd, const hc_hit* __restrict__ sb, const int32_t* __restrict__ sg, const int32_t* __restrict__ sc,
    const int32_t* __restrict__ si, hc_hit* db, int32_t* dg, int32_t* dc, int32_t* di,
    const hc_features* __restrict__ f, const int32_t* __restrict__ cmin, hc_features* q, int64_t q_cap, int nb_grid)
{
    constexpr int PER = kCmpBlock / kCmpThreads;
    const int n = sd->n_all;
    const int nb = (n + kCmpBlock - 1) / kCmpBlock;
    if (sd->n_clusters < 0 || nb == 0) {  // nothing to move
        if (blockIdx.x == 0 && threadIdx.x == 0) end_push(sd);
        return;
    }
    const int g = (int)blockIdx.x;
    const bool rows = g >= nb_grid;
    const int b = rows ? (g - nb_grid) / PER : g;
    if (b >= nb || nb > nb_grid) return;  // beyond this push (nb <= nb_grid: the grid's bound)
    if (!rows) {
        flag_scatter(keep, n, b, hoff[b], 0, PER, [&](int64_t i, uint64_t p) {
            db[p] = sb[i];
            dg[p] = sg[i];
            dc[p] = sc[i];
            if (si) di[p] = si[i];
        });
        if (last_group(sd, (uint32_t)nb) && threadIdx.x == 0) end_push(sd);
    } else {
        const int slice = (g - nb_grid) % PER;
        const int K = sd->n_clusters;
        if ((int64_t)b * kCmpBlock + (int64_t)slice * kCmpThreads < K) {  // rows from K on are never flagged
            const int64_t tmod = sd->q_base % q_cap;
            flag_scatter(fflag, n, b, foff[b], slice, slice + 1, [&](int64_t k, uint64_t p) {
                hc_features r = f[k];
                r.label = cmin ? cmin[k] : sg[r.label];  // row k is the cluster of rank k
                int64_t x = tmod + (int64_t)p;
                if (x >= q_cap) x %= q_cap;
                q[x] = r;
            });
        }
    }
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
    int k = 0;              // chunks of the push (0 for a flush)
    int slot[kMaxPushChunks];
    uint64_t tag[kMaxPushChunks];
    int32_t n = 0;          // their hits
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
    // device state block: the state, then the chunk table
    char* state = nullptr;
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
    (void)hipFree(st->state);
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
    const ChunkRec* cr = reinterpret_cast<const ChunkRec*>(r->mirror + kStateHdr);
    if (d.n_clusters < 0) st->failed = true;
    for (int j = 0; j < r->k; j++)
        if (cr[r->slot[j]].verdict != HC_OK) {
            ChunkHost& c = st->chunks[r->slot[j]];
            st->done.emplace_back(c.tag, cr[r->slot[j]].verdict);
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
    if (st->log_retired)  // the push's closed clusters count for its last chunk
        for (int j = 0; j < r->k; j++)
            st->retired_log.push_back(
                RetiredPush{r->tag[j], cr[r->slot[j]].verdict, j == r->k - 1 ? d.n_closed : 0, j == r->k - 1});
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
        if ((rc = dev_alloc(&st->flags, 2 * nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->lab, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->feats, nc)) != HC_OK) return rc;
        if ((rc = dev_alloc(&st->counts, 2 * count_slots(nc))) != HC_OK) return rc;
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
    const size_t per_hit = 2 * (sizeof(hc_hit) + 4 + 4) + 2 + 4 + sizeof(hc_features) + (ids ? 3 * 4 : 0);
    return (size_t)cap * per_hit + 4 * 2 * (size_t)count_slots(cap) + ws + sizeof(hc_features) * (size_t)q +
           sizeof(ChunkRec) * (size_t)chunks + kStateHdr;
}

// The state block with room for twice the chunk slots (64 at first): the
// state and the table so far are carried over, a new stream's state is zero.
static int grow_chunks(hc_stream* st)
{
    hipError_t e;
    int rc = reap(st, true);
    if (rc != HC_OK) return rc;
    const int nc = st->chunk_cap ? st->chunk_cap * 2 : 64;
    char* d;
    if ((rc = dev_alloc(&d, kStateHdr + sizeof(ChunkRec) * (size_t)nc)) != HC_OK) return rc;
    if (st->state)
        e = hipMemcpyAsync(d, st->state, kStateHdr + sizeof(ChunkRec) * (size_t)st->chunk_cap, hipMemcpyDeviceToDevice,
                           st->s);
    else
        e = hipMemsetAsync(d, 0, kStateHdr, st->s);
    if (e == hipSuccess) e = hipStreamSynchronize(st->s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return set_device_error(e, "stream chunk table");
    }
    (void)hipFree(st->state);
    st->state = d;
    st->sd = reinterpret_cast<StreamDev*>(d);
    st->chunks_dev = reinterpret_cast<ChunkRec*>(d + kStateHdr);
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
    const size_t need = kStateHdr + sizeof(ChunkRec) * (size_t)st->chunk_cap;
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

// Enqueue one push of the chunks pc (k = 0: a flush, the closing of every
// open cluster): append + commit, the plain clustering over the
// device-resident count, closing and compaction, then the pinned read-back of
// state and chunk table.
static int enqueue_push(hc_stream* st, const hc_hit* hits, const int32_t* in_ids, const PushChunks& pc,
                        const uint64_t* tags, int64_t n_all_bound)
{
    const int32_t n = pc.start[pc.k];
    const int nb_in = (n + kAppendBlock - 1) / kAppendBlock;
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
        if (pc.k == 0) {
            hipLaunchKernelGGL(k_stream_commit_flush, dim3(1), dim3(64), 0, st->s, st->sd, st->dt);
        } else if (pc.k == 1) {  // n > 0: a chunk of nothing never gets here
            hipLaunchKernelGGL(k_stream_append, dim3(nb_in), dim3(256), 0, st->s, hits, in_ids, pc, st->buf[st->cur],
                               st->gidx[st->cur], st->ids[st->cur], st->cslot[st->cur], st->sd, st->chunks_dev,
                               st->tdis, st->W, st->H);
        } else {
            hipLaunchKernelGGL(k_stream_chunk_stats, dim3(nb_in), dim3(256), 0, st->s, hits, in_ids, pc, st->sd,
                               st->chunks_dev, st->id_mode == 1 ? 1 : 0, st->tdis, st->W, st->H);
            hipLaunchKernelGGL(k_stream_place, dim3(nb_in), dim3(256), 0, st->s, hits, in_ids, pc, st->sd,
                               st->buf[st->cur], st->gidx[st->cur], st->ids[st->cur], st->cslot[st->cur]);
        }
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
            // keep/flag bytes and per-block counts: hits in the first half, feature rows in the second
            uint8_t* fflag = st->flags + st->cap;
            uint32_t* fcount = st->counts + count_slots(st->cap);
            hipLaunchKernelGGL(k_stream_close, dim3(nb), dim3(kCloseThreads), 0, st->s, st->lab, w, st->gidx[st->cur],
                               st->cslot[st->cur], cmin, st->feats, st->chunks_dev, st->sd, st->dt, pc.k == 0, st->flags,
                               fflag, st->counts, fcount);
            hipLaunchKernelGGL(k_stream_scatter, dim3(nb * (1 + kCmpBlock / kCmpThreads)), dim3(kCmpThreads), 0, st->s,
                               st->flags, fflag, st->counts, fcount, st->sd, st->buf[st->cur], st->gidx[st->cur],
                               st->cslot[st->cur], st->ids[st->cur], st->buf[nxt], st->gidx[nxt], st->cslot[nxt],
                               st->ids[nxt], st->feats, cmin, st->queue, st->q_cap, nb);
        }
        if ((e = hipGetLastError()) != hipSuccess) return give_back(set_device_error(e, "stream close"));
    }
    if ((e = hipMemcpyAsync(r->mirror, st->state, kStateHdr + sizeof(ChunkRec) * st->chunk_cap, hipMemcpyDeviceToHost,
                            st->s)) != hipSuccess ||
        (e = hipEventRecord(r->ev, st->s)) != hipSuccess)
        return give_back(set_device_error(e, "stream read-back"));
    r->seq = st->seq++;
    r->k = pc.k;
    r->n = n;
    r->mirror_chunks = st->chunk_cap;
    st->inflight.push_back(r);
    for (int j = 0; j < pc.k; j++) {
        r->slot[j] = pc.slot[j];
        r->tag[j] = tags[j];
        ChunkHost& c = st->chunks[pc.slot[j]];
        c.tag = tags[j];
        c.reg_seq = r->seq;
        c.active = true;
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
    int rc = HC_OK;
    if ((e = hipStreamCreateWithFlags(&st->ds, hipStreamNonBlocking)) != hipSuccess)
        rc = set_device_error(e, "hipStreamCreate");
    if (rc == HC_OK) rc = grow_chunks(st);  // the state block, zeroed
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

// One push of k chunks stored back to back at hits (and ids), chunk j with
// counts[j] hits, labels[j] and tags[j].
static int push_chunks(hc_stream* st, const hc_hit* hits, const int32_t* ids, int k, const int32_t* counts,
                       int32_t* const* labels, const uint64_t* tags)
{
    if (!st) return set_error(HC_ERR_ARG, "stream is NULL");
    if (st->failed) return set_error(HC_ERR_DEVICE, "stream failed earlier");
    if (k < 1 || k > kMaxPushChunks || !counts) return set_error(HC_ERR_ARG, "bad chunk list");
    int64_t n = 0;
    for (int j = 0; j < k; j++) {
        if (counts[j] < 0 || (counts[j] > 0 && !labels[j])) return set_error(HC_ERR_ARG, "bad chunk arguments");
        if (k > 1 && counts[j] == 0) return set_error(HC_ERR_ARG, "an empty chunk in a push of several");
        n += counts[j];
    }
    if (n > 0 && (!hits || (st->id_mode == 1 && !ids))) return set_error(HC_ERR_ARG, "bad chunk arguments");
    const int mode = ids ? 1 : 0;
    if (n > 0 && st->id_mode >= 0 && st->id_mode != mode)
        return set_error(HC_ERR_ARG, "a stream takes ids with every push or with none");
    if (st->pushed + n > 0x7FFFFFFF) return set_error(HC_ERR_OVERFLOW, "more than 2^31 - 1 hits in the stream");
    if (n == 0) {
        st->done.emplace_back(tags[0], HC_OK);
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
    PushChunks pc{};
    pc.k = k;
    for (int j = 0, c = 0; j < k; j++) {
        for (;;) {
            while (c < st->chunk_cap && st->chunks[c].active) c++;
            if (c < st->chunk_cap) break;
            if ((rc = grow_chunks(st)) != HC_OK) return rc;
        }
        pc.slot[j] = c++;
        pc.start[j + 1] = pc.start[j] + counts[j];
        pc.labels[j] = labels[j];
    }
    if ((rc = ensure_capacity(st, open_bound(st) + n)) != HC_OK) return rc;
    if ((rc = ensure_queue(st, open_bound(st) + n)) != HC_OK) return rc;
    // a growth above may have waited for the pushes in flight, which tightens
    // the bound and changes the sort hint: size the workspace for the final plan
    const int64_t n_all = open_bound(st) + n;
    if ((rc = ensure_capacity(st, n_all)) != HC_OK) return rc;
    if ((rc = enqueue_push(st, hits, ids, pc, tags, n_all)) != HC_OK) return rc;
    st->pushed += n;
    return HC_OK;
}

static int push_impl(hc_stream* st, const hc_hit* hits, const int32_t* ids, int32_t n, int32_t* labels,
                     uint64_t tag)
{
    return push_chunks(st, hits, ids, 1, &n, &labels, &tag);
}

int hc_stream_push_chunks(hc_stream* st, const hc_hit* hits, int32_t k, const int32_t* counts,
                          int32_t* const* labels, const uint64_t* tags)
{
    if (k < 1 || k > kMaxPushChunks || !counts || !labels || !tags) return set_error(HC_ERR_ARG, "bad chunk list");
    return push_chunks(st, hits, nullptr, k, counts, labels, tags);
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
    const PushChunks none{};  // k = 0: a flush
    if ((rc = enqueue_push(st, nullptr, nullptr, none, nullptr, n_all)) != HC_OK) return rc;
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
