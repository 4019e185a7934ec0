// The paper's second cluster definition, Section 2 (iii)(b): a cluster is a
// maximal set of hits that is spatially connected (8-neighbouring or
// identical pixels, any ToA) and whose ToAs, in order, leave no gap larger
// than dt (every hit but the earliest has another within dt before it).
// Maximal under inclusion, these sets partition the hits; every (iii)(a)
// cluster lies inside one of them.
//
// After the usual ToA ordering (step A1), the parts of a partition are
// refined on the device until they no longer change, starting from one part
// holding every hit:
//   1. the positions are sorted stably by part (ToA order inside a part) and
//      every part is cut where its ToA jumps by more than dt; a segment is
//      named by the sorted position of its first hit (a max-scan of the
//      boundary positions);
//   2. the positions are sorted by (segment, pixel); every hit is joined
//      (union-find) to the first hit of its segment at each of its 9 pixels,
//      found by galloping from its own place in that order; the new part of
//      a hit is its component's root.
// A set that is spatially connected and gap-free never straddles a cut of
// either kind, so it stays inside one part; when a round leaves the number
// of parts unchanged (parts only split), every part is connected and
// gap-free, i.e. a cluster.  The host reads the count after every round.
// The cluster's label -- its smallest input index -- is then published in
// the input-index forest, and the feature stages run unchanged.
#include <algorithm>

#include "hc_device.h"
#include "hc_radix.h"

namespace hc {

constexpr int kGlbThreads = 256;
constexpr int kGlbScanBlock = 1024;  // positions per max-scan block (4 per thread)

struct GlbWork {
    int32_t* part;      // per sorted position: its part (a position of the part)
    int32_t* seg;       // per sorted position: its segment
    int32_t* order;     // positions in (part, ToA) order, then in (segment, pixel) order
    uint64_t* keys;     // segment * pixels + pixel, in (segment, pixel) order
    int32_t* scan;      // boundary positions, max-scanned
    int32_t* bmax;      // per scan block
    int32_t* par;       // union-find forest over positions
    int32_t* minidx;    // per root position: smallest input index of the part
    int32_t* count;     // parts after the round ([0]), error flag ([1])
    int32_t n_scan_blocks;
};

// -------------------------------------------------------------- sort jobs
// Stable radix sorts on the fallback engine: every job ends by writing the
// values (and keys) in sorted order itself.
struct PartSortJob {
    static constexpr bool kKeepSorted = false;
    Work w;
    GlbWork g;
    __device__ int64_t count() const { return w.n; }
    __device__ void load(int64_t j, uint64_t& k, uint32_t& v) const
    {
        k = (uint64_t)(uint32_t)g.part[j];
        v = (uint32_t)j;
    }
    __device__ int plan(RadixState& st, RadixLds&)
    {
        if (threadIdx.x == 0) {
            st.active = 1;
            st.key_min = 0;
            const uint32_t top = (uint32_t)(w.n - 1);
            const int bits = top == 0 ? 0 : 32 - __builtin_clz(top);
            st.passes = bits <= 8 ? 1 : (bits + 7) / 8;
        }
        return 0;
    }
    __device__ void store(int64_t pos, uint64_t, uint32_t v) const { g.order[pos] = (int32_t)v; }
    __device__ void extra(int, const uint64_t*, const uint32_t*, RadixLds&) {}
};

__device__ inline uint32_t pixel_of(uint32_t xy, uint32_t W) { return (xy >> 16) * W + (xy & 0xFFFFu); }

struct SegPixSortJob {
    static constexpr bool kKeepSorted = false;
    Work w;
    GlbWork g;
    __device__ int64_t count() const { return w.n; }
    __device__ void load(int64_t p, uint64_t& k, uint32_t& v) const
    {
        const uint64_t npix = (uint64_t)w.width * w.height;
        k = (uint64_t)(uint32_t)g.seg[p] * npix + pixel_of(w.s_xy[p], w.width);
        v = (uint32_t)p;
    }
    __device__ int plan(RadixState& st, RadixLds&)
    {
        if (threadIdx.x == 0) {
            st.active = 1;
            st.key_min = 0;
            const uint64_t top = (uint64_t)(w.n - 1) * ((uint64_t)w.width * w.height) + (uint64_t)w.width * w.height - 1;
            const int bits = top == 0 ? 0 : 64 - __builtin_clzll(top);
            st.passes = bits <= 8 ? 1 : (bits + 7) / 8;
        }
        return 0;
    }
    __device__ void store(int64_t pos, uint64_t key, uint32_t v) const
    {
        g.keys[pos] = key;
        g.order[pos] = (int32_t)v;
    }
    __device__ void extra(int, const uint64_t*, const uint32_t*, RadixLds&) {}
};

__global__ void k_glb_reset_sort(Work w)
{
    int32_t* s = reinterpret_cast<int32_t*>(&w.status->rs[1]);
    for (int i = threadIdx.x; i < (int)(sizeof(RadixState) / 4); i += blockDim.x) s[i] = 0;
}

template <class Job>
__global__ __launch_bounds__(kFbThreads) void k_glb_sort(Work w, GlbWork g)
{
    if (w.status->err_range || g.count[1]) return;
    Job job{w, g};
    uint64_t* kb[2] = {w.fb_key[0], w.fb_key[1]};
    uint32_t* vb[2] = {w.fb_val[0], w.fb_val[1]};
    radix_engine(job, &w.status->rs[1], kb, vb, w.fb_hist, w.n_fb_blocks, &w.status->err_internal);
}

// --------------------------------------------------------------- rounds
__global__ __launch_bounds__(kGlbThreads) void k_glb_init(Work w, GlbWork g)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < w.n; p += (int64_t)gridDim.x * blockDim.x)
        g.part[p] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.count[0] = 1;
        g.count[1] = 0;
    }
}

// boundary positions of the ToA segments in (part, ToA) order (-1 elsewhere)
__global__ __launch_bounds__(kGlbThreads) void k_glb_bounds(Work w, GlbWork g)
{
    if (w.status->err_range || g.count[1]) return;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < w.n; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = g.order[j];
        bool b = j == 0;
        if (!b) {
            const int32_t q = g.order[j - 1];
            b = g.part[p] != g.part[q] || w.s_toa[p] - w.s_toa[q] > w.dt;
        }
        g.scan[j] = b ? (int32_t)j : -1;
    }
}

// inclusive max-scan of g.scan: per block, block maxima, then the carry
__device__ inline int32_t wave_incl_max(int32_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t u = __shfl_up(v, o, kWave);
        if (lane >= o) v = u > v ? u : v;
    }
    return v;
}

__global__ __launch_bounds__(kGlbThreads) void k_glb_scan_local(Work w, GlbWork g)
{
    __shared__ int32_t wmax[kGlbThreads / kWave];
    constexpr int PER = kGlbScanBlock / kGlbThreads;
    if (w.status->err_range || g.count[1]) return;
    const int64_t j0 = (int64_t)blockIdx.x * kGlbScanBlock + (int64_t)threadIdx.x * PER;
    int32_t v[PER];
    int32_t run = -1;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        v[q] = j0 + q < w.n ? g.scan[j0 + q] : -1;
        run = v[q] > run ? v[q] : run;
        v[q] = run;
    }
    const int32_t incl = wave_incl_max(run);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == kWave - 1) wmax[wid] = incl;
    __syncthreads();
    int32_t before = __shfl_up(incl, 1, kWave);
    if (lane == 0) before = -1;
    for (int k = 0; k < wid; k++) before = wmax[k] > before ? wmax[k] : before;
#pragma unroll
    for (int q = 0; q < PER; q++)
        if (j0 + q < w.n) g.scan[j0 + q] = v[q] > before ? v[q] : before;
    if (threadIdx.x == kGlbThreads - 1) {
        int32_t m = incl;
        for (int k = 0; k < wid; k++) m = wmax[k] > m ? wmax[k] : m;
        g.bmax[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(1024) void k_glb_scan_blocks(Work w, GlbWork g)
{
    __shared__ int32_t wmax[1024 / kWave];
    if (w.status->err_range || g.count[1]) return;
    int32_t carry = -1;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int c0 = 0; c0 < g.n_scan_blocks; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int32_t v = i < g.n_scan_blocks ? g.bmax[i] : -1;
        const int32_t incl = wave_incl_max(v);
        if (lane == kWave - 1) wmax[wid] = incl;
        __syncthreads();
        int32_t before = __shfl_up(incl, 1, kWave);
        if (lane == 0) before = -1;
        for (int k = 0; k < wid; k++) before = wmax[k] > before ? wmax[k] : before;
        before = carry > before ? carry : before;
        if (i < g.n_scan_blocks) g.bmax[i] = before;  // exclusive: the maximum of the earlier blocks
        int32_t total = -1;
        for (int k = 0; k < 1024 / kWave; k++) total = wmax[k] > total ? wmax[k] : total;
        carry = total > carry ? total : carry;
        __syncthreads();
    }
}

// segment of every position: the last boundary at or before it
__global__ __launch_bounds__(kGlbThreads) void k_glb_segments(Work w, GlbWork g)
{
    if (w.status->err_range || g.count[1]) return;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < w.n; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = g.bmax[j / kGlbScanBlock];
        int32_t s = g.scan[j];
        s = c > s ? c : s;
        if (s < 0 || s > j) {
            atomicOr(&w.status->err_internal, 1);
            s = 0;
        }
        g.seg[g.order[j]] = s;
        g.par[j] = (int32_t)j;  // fresh forest for the spatial step
    }
}

// first place in keys[0..n) with key >= target, galloping from j
__device__ inline int64_t gallop_lower(const uint64_t* keys, int64_t n, int64_t j, uint64_t target)
{
    int64_t lo, hi;
    if (keys[j] < target) {
        lo = j + 1;
        int64_t step = 1;
        hi = lo;
        while (hi < n && keys[hi] < target) {
            lo = hi + 1;
            hi += step;
            step <<= 1;
        }
        if (hi > n) hi = n;
    } else {
        hi = j;
        int64_t step = 1;
        lo = hi - 1;
        while (lo >= 0 && keys[lo] >= target) {
            hi = lo;
            lo -= step;
            step <<= 1;
        }
        if (lo < 0) lo = 0;
    }
    while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (keys[m] < target) lo = m + 1; else hi = m;
    }
    return lo;
}

// spatial components inside every segment: join each hit to the first hit
// of its segment at each of its 9 pixels (places in (segment, pixel) order)
__global__ __launch_bounds__(kGlbThreads) void k_glb_link(Work w, GlbWork g)
{
    if (w.status->err_range || g.count[1]) return;
    const uint64_t npix = (uint64_t)w.width * w.height;
    const int64_t n = w.n;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = g.keys[j];
        const uint64_t s = key / npix;
        const uint32_t pix = (uint32_t)(key - s * npix);
        const int x = (int)(pix % w.width), y = (int)(pix / w.width);
        for (int dy = -1; dy <= 1; dy++) {
            const int qy = y + dy;
            if (qy < 0 || qy >= (int)w.height) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int qx = x + dx;
                if (qx < 0 || qx >= (int)w.width) continue;
                const uint64_t t = s * npix + (uint64_t)qy * w.width + (uint64_t)qx;
                const int64_t f = gallop_lower(g.keys, n, j, t);
                if (f < n && g.keys[f] == t && f != j) gunion(g.par, (int32_t)f, (int32_t)j, &w.status->err_internal);
            }
        }
    }
}

// new parts: every position takes the root of its component (a place in
// (segment, pixel) order, mapped back to a sorted position); count roots
__global__ __launch_bounds__(kGlbThreads) void k_glb_parts(Work w, GlbWork g, int32_t* round_count)
{
    __shared__ int32_t bc;
    if (threadIdx.x == 0) bc = 0;
    __syncthreads();
    const bool stop = w.status->err_range || g.count[1];
    int32_t c = 0;
    if (!stop) {
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < w.n;
             j += (int64_t)gridDim.x * blockDim.x) {
            const int32_t r = gfind_final(g.par, (int32_t)j, &w.status->err_internal);
            g.part[g.order[j]] = g.order[r];
            c += r == (int32_t)j;
        }
    }
    if (c) atomicAdd(&bc, c);
    __syncthreads();
    if (threadIdx.x == 0 && bc) atomicAdd(round_count, bc);
}

__global__ void k_glb_round_begin(GlbWork g, int32_t* round_count)
{
    if (threadIdx.x == 0) *round_count = 0;
}

// end of a round: the count and whether anything went wrong
__global__ void k_glb_round_end(Work w, GlbWork g, const int32_t* round_count, int32_t* host_view)
{
    if (threadIdx.x != 0) return;
    const bool bad = w.status->err_range || w.status->err_internal || g.count[1];
    if (bad) g.count[1] = 1;
    host_view[0] = bad ? -1 : *round_count;
    host_view[1] = g.count[0];
    g.count[0] = *round_count;
}

// labels: the smallest input index of every part, published as the parent
// of each of its hits in the input-index forest that the flatten pass reads
__global__ __launch_bounds__(kGlbThreads) void k_glb_min_init(Work w, GlbWork g)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < w.n; p += (int64_t)gridDim.x * blockDim.x)
        g.minidx[p] = 0x7FFFFFFF;
}

__global__ __launch_bounds__(kGlbThreads) void k_glb_min(Work w, GlbWork g)
{
    if (w.status->err_range) return;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < w.n; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = g.part[p];
        if (r < 0 || r >= w.n) {
            atomicOr(&w.status->err_internal, 1);
            continue;
        }
        atomicMin(&g.minidx[r], w.s_idx[p]);
    }
}

__global__ __launch_bounds__(kGlbThreads) void k_glb_publish(Work w, GlbWork g)
{
    if (w.status->err_range) return;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < w.n; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = g.part[p];
        const int32_t i = w.s_idx[p];
        if (r < 0 || r >= w.n || i < 0 || i >= w.n) {
            atomicOr(&w.status->err_internal, 1);
            continue;
        }
        w.gparent[i] = g.minidx[r];
    }
}

// ------------------------------------------------------------ host side
static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

size_t plan_global(int64_t n, GlbWork* g, char* base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += up256(bytes);
        return p;
    };
    const size_t N = (size_t)(n > 0 ? n : 1);
    GlbWork x{};
    x.n_scan_blocks = (int32_t)((N + kGlbScanBlock - 1) / kGlbScanBlock);
    x.part = (int32_t*)take(4 * N);
    x.seg = (int32_t*)take(4 * N);
    x.order = (int32_t*)take(4 * N);
    x.keys = (uint64_t*)take(8 * N);
    x.scan = (int32_t*)take(4 * N);
    x.bmax = (int32_t*)take(4 * (size_t)x.n_scan_blocks);
    x.par = (int32_t*)take(4 * N);
    x.minidx = (int32_t*)take(4 * N);
    x.count = (int32_t*)take(16);
    if (g) *g = x;
    return off;
}

// The (iii)(b) clustering on a planned workspace: ordering, refinement rounds
// (the host waits for each round's count), labels, features.  host_view: 2
// pinned int32 for the round counts.
int enqueue_cluster_global(const hc_hit* hits, const Work& w, const GlbWork& g, int32_t* labels,
                           hc_features* features, int32_t* n_clusters, int32_t* host_view, hipStream_t s)
{
    hipError_t e;
#define HC_LAUNCH(call, what)                                                       \
    do {                                                                            \
        if ((e = (call)) != hipSuccess) return set_device_error(e, what);           \
    } while (0)
#define HC_KERNEL(...)                                                              \
    do {                                                                            \
        hipLaunchKernelGGL(__VA_ARGS__);                                            \
        if ((e = hipGetLastError()) != hipSuccess) return set_device_error(e, "global-time round"); \
    } while (0)
    HC_LAUNCH(launch_init(w, s), "init");
    HC_LAUNCH(launch_tile_sort(hits, w, s), "tile_sort");
    if (!w.force_fallback) HC_LAUNCH(launch_tile_merge(w, s), "tile_merge");
    HC_LAUNCH(launch_sort_fallback(hits, w, s), "sort_fallback");
    const int grid = (int)std::min<int64_t>(((int64_t)w.n + kGlbThreads - 1) / kGlbThreads, 8192);
    const int pg = persistent_grid();
    TimedLaunch tl("global_rounds", s);
    HC_KERNEL(k_glb_init, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
    int32_t* round_count = g.count + 2;
    for (;;) {  // every round that does not end it splits a part: at most n rounds
        HC_KERNEL(k_glb_reset_sort, dim3(1), dim3(256), 0, s, w);
        HC_KERNEL(k_glb_sort<PartSortJob>, dim3(pg), dim3(kFbThreads), 0, s, w, g);
        HC_KERNEL(k_glb_bounds, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
        HC_KERNEL(k_glb_scan_local, dim3(g.n_scan_blocks), dim3(kGlbThreads), 0, s, w, g);
        HC_KERNEL(k_glb_scan_blocks, dim3(1), dim3(1024), 0, s, w, g);
        HC_KERNEL(k_glb_segments, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
        HC_KERNEL(k_glb_reset_sort, dim3(1), dim3(256), 0, s, w);
        HC_KERNEL(k_glb_sort<SegPixSortJob>, dim3(pg), dim3(kFbThreads), 0, s, w, g);
        HC_KERNEL(k_glb_link, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
        HC_KERNEL(k_glb_round_begin, dim3(1), dim3(64), 0, s, g, round_count);
        HC_KERNEL(k_glb_parts, dim3(grid), dim3(kGlbThreads), 0, s, w, g, round_count);
        HC_KERNEL(k_glb_round_end, dim3(1), dim3(64), 0, s, w, g, round_count, host_view);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return set_device_error(e, "global-time round");
        const int32_t now = host_view[0], before = host_view[1];
        if (now < 0) break;       // an error: the count kernels report it
        if (now == before) break; // nothing split: the parts are the clusters
    }
    HC_KERNEL(k_glb_min_init, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
    HC_KERNEL(k_glb_min, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
    HC_KERNEL(k_glb_publish, dim3(grid), dim3(kGlbThreads), 0, s, w, g);
    HC_LAUNCH(launch_flatten(w, labels, s), "flatten");
    HC_LAUNCH(launch_scan_blocks(w, n_clusters, s), "scan_blocks");
    if (features) {
        HC_LAUNCH(launch_features(w, labels, s), "features");
        HC_LAUNCH(launch_carries(w, s), "carries");
        HC_LAUNCH(launch_compact(w, features, s), "compact");
    }
#undef HC_KERNEL
#undef HC_LAUNCH
    return HC_OK;
}

// Pinned words the host reads after every round (one pair per host thread).
static int32_t* round_view()
{
    static thread_local int32_t* v = nullptr;
    if (!v && hipHostMalloc((void**)&v, 4 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) v = nullptr;
    return v;
}

int global_cluster(const hc_hit* hits, Work& w, char* extra, int32_t* labels, hc_features* features,
                   int32_t* n_clusters, hipStream_t s)
{
    GlbWork g;
    plan_global(w.n, &g, extra);
    int32_t* view = round_view();
    if (!view) return set_error(HC_ERR_DEVICE, "hipHostMalloc(round counts)");
    return enqueue_cluster_global(hits, w, g, labels, features, n_clusters, view, s);
}

}  // namespace hc
