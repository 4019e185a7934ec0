// Steps A2 and A3 of the clustering path: neighbour search and union-find.
//
// The paper (Section 4.1) sweeps the ToA-sorted hits, finds for each hit the
// latest earlier hit at each of "the 8 neighbouring pixels plus the pixel
// itself" through a per-pixel matrix, and joins the clusters with union-find.
// Its GPU version gives every thread one chunk and one full 256 x 256 matrix.
//
// Here each work-group takes a tile of kLinkTile consecutive sorted hits plus
// the "halo" of earlier hits whose ToA lies within dt of the tile's first hit,
// and works entirely in LDS:
//   * a pixel hash (open addressing) maps each occupied pixel of the tile and
//     halo to the list of its hits -- the tile-sized replacement of the
//     paper's dense matrix;
//   * each tile hit b probes its 9 pixels and joins ONE earlier hit at each
//     pixel that is within dt of it.  Any such hit will do: the hits of one
//     pixel whose consecutive ToAs differ by <= dt are already chained by
//     their own-pixel probes, so joining any of them joins the one the
//     paper's "latest hit" rule would have picked;
//   * joins go into an LDS union-find that links the root with the larger
//     input index under the smaller one, so every tree's root is its smallest
//     input index -- the canonical label;
//   * the tile's forest is written to the global parent array; halo hits that
//     the tile joined together are queued as cross-tile edges.
// A tile whose halo does not fit (or whose ToA span exceeds 32 bits) is
// handled by k_link_fallback: a pixel-sorted copy of all hits plus binary
// searches.  k_union_edges applies the queued cross-tile edges with atomic
// compare-and-swap, and k_flatten writes labels[i] = root(i).
#include "hc_device.h"
#include "hc_radix.h"

namespace hc {

__device__ inline uint32_t pix_hash(uint32_t key) { return (key * 0x9E3779B1u) >> 20; }  // 12 bits

// ---- LDS union-find over local slots, roots = smallest input index
__device__ inline int32_t ld_lds(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void st_lds(int32_t* p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline int32_t lfind(int32_t* par, int32_t x)
{
    while (true) {
        const int32_t p = ld_lds(par + x);
        if (p == x) return x;
        const int32_t g = ld_lds(par + p);
        if (g != p) st_lds(par + x, g);
        x = g;
    }
}

__device__ inline void lunion(int32_t* par, const int32_t* idx, int32_t a, int32_t b)
{
    while (true) {
        a = lfind(par, a);
        b = lfind(par, b);
        if (a == b) return;
        if (idx[a] > idx[b]) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        int32_t expected = b;
        if (__hip_atomic_compare_exchange_strong(par + b, &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
    }
}

__global__ __launch_bounds__(kLinkThreads) void k_link(Work w)
{
    constexpr int LCAP = kLinkTile + kLinkHaloCap;
    __shared__ uint32_t l_toa[LCAP];
    __shared__ uint32_t l_xy[LCAP];
    __shared__ int32_t l_idx[LCAP];
    __shared__ int32_t l_par[LCAP];
    __shared__ int16_t l_next[LCAP];
    __shared__ uint32_t h_key[kLinkHash];
    __shared__ int32_t h_head[kLinkHash];
    __shared__ int64_t s_h0;
    __shared__ int s_overflow;

    if (w.status->err_range) return;
    const int tile = xcd_tile(w.n_link_tiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)tile * kLinkTile;
    const int64_t p1 = (p0 + kLinkTile) < w.n ? (p0 + kLinkTile) : w.n;

    // ---- halo: earlier hits with toa >= toa(first) - dt (a suffix of the
    // sorted positions before p0), searched backwards 64 at a time
    if (t < kWave) {
        const uint64_t lo = sat_sub_u64(w.s_toa[p0], w.dt);
        const int64_t lim = p0 - kLinkHaloCap > 0 ? p0 - kLinkHaloCap : 0;
        int64_t c = p0, h0 = p0;
        while (c > lim) {
            const int64_t cs = c - kWave > lim ? c - kWave : lim;
            const int64_t q = c - kWave + t;
            const bool in = q >= cs && w.s_toa[q] >= lo;
            const int nin = __popcll(__ballot(in));
            h0 = c - nin;
            if (nin < c - cs) break;
            c = cs;
        }
        bool overflow = (h0 == lim && lim > 0 && w.s_toa[lim - 1] >= lo);
        overflow |= (w.s_toa[p1 - 1] - w.s_toa[h0]) > 0xFFFFFFFFull;
        if (t == 0) {
            s_h0 = h0;
            s_overflow = overflow ? 1 : 0;
        }
    }
    __syncthreads();
    const int64_t h0 = s_h0;
    if (s_overflow) {
        for (int64_t p = p0 + t; p < p1; p += kLinkThreads) {
            const int32_t id = w.s_idx[p];
            if (id >= 0 && id < w.n) w.gparent[id] = id;
            else atomicOr(&w.status->err_internal, 1);
        }
        if (t == 0) {
            const int k = atomicAdd(&w.status->n_overflow, 1);
            w.overflow_tiles[k] = tile;
        }
        return;
    }
    const int L = (int)(p1 - h0);
    const int hl = (int)(p0 - h0);
    const uint64_t tbase = w.s_toa[h0];
    for (int i = t; i < L; i += kLinkThreads) {
        const int64_t p = h0 + i;
        l_toa[i] = (uint32_t)(w.s_toa[p] - tbase);
        l_xy[i] = w.s_xy[p];
        int32_t id = w.s_idx[p];
        if (id < 0 || id >= w.n) {
            atomicOr(&w.status->err_internal, 1);
            id = 0;
        }
        l_idx[i] = id;
        l_par[i] = i;
    }
    for (int i = t; i < kLinkHash; i += kLinkThreads) {
        h_key[i] = 0u;
        h_head[i] = -1;
    }
    __syncthreads();

    // ---- pixel hash: slot per occupied pixel, list of its hits
    for (int i = t; i < L; i += kLinkThreads) {
        const uint32_t key = l_xy[i] + 1u;
        uint32_t slot = pix_hash(key);
        while (true) {
            const uint32_t old = atomicCAS(&h_key[slot], 0u, key);
            if (old == 0u || old == key) break;
            slot = (slot + 1u) & (kLinkHash - 1);
        }
        l_next[i] = (int16_t)atomicExch(&h_head[slot], i);
    }
    __syncthreads();

    // ---- neighbour search of the tile hits
    const uint64_t dt = w.dt;
    const int W = (int)w.width, H = (int)w.height;
    for (int i = hl + t; i < L; i += kLinkThreads) {
        const uint32_t xy = l_xy[i];
        const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
        const uint32_t ti = l_toa[i];
        for (int dy = -1; dy <= 1; dy++) {
            const int qy = y + dy;
            if (qy < 0 || qy >= H) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int qx = x + dx;
                if (qx < 0 || qx >= W) continue;
                const uint32_t key = ((uint32_t)qx | ((uint32_t)qy << 16)) + 1u;
                uint32_t slot = pix_hash(key);
                int a = -1;
                while (true) {
                    const uint32_t k = h_key[slot];
                    if (k == key) {
                        a = h_head[slot];
                        break;
                    }
                    if (k == 0u) break;
                    slot = (slot + 1u) & (kLinkHash - 1);
                }
                while (a >= 0) {
                    if (a < i && (uint64_t)(ti - l_toa[a]) <= dt) {
                        lunion(l_par, l_idx, a, i);
                        break;
                    }
                    a = l_next[a];
                }
            }
        }
    }
    __syncthreads();
    for (int i = t; i < L; i += kLinkThreads) st_lds(l_par + i, lfind(l_par, i));
    __syncthreads();

    // ---- publish: tile hits get their local root, joined halo hits become edges
    for (int i = t; i < L; i += kLinkThreads) {
        const int32_t r = l_par[i];
        if (i >= hl) {
            w.gparent[l_idx[i]] = l_idx[r];
        } else if (r != i) {
            const int e = atomicAdd(&w.status->n_edges, 1);
            if (e < w.edge_cap) w.edges[e] = make_int2(l_idx[i], l_idx[r]);
            else atomicOr(&w.status->err_internal, 1);
        }
    }
}

hipError_t launch_link(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link", s);
    hipLaunchKernelGGL(k_link, dim3(xcd_grid(w.n_link_tiles)), dim3(kLinkThreads), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------- link fallback (big halos)
// Hits sorted by (pixel, sorted position); for each hit of an overflowed
// tile and each of its 9 pixels, the latest earlier hit at that pixel is
// found by binary search and joined if within dt.
struct PixSortJob {
    static constexpr bool kKeepSorted = true;
    Work w;
    __device__ int64_t count() const { return w.n; }
    __device__ void load(int64_t i, uint64_t& k, uint32_t& v) const
    {
        const uint32_t xy = w.s_xy[i];
        k = (uint64_t)(xy >> 16) * w.width + (xy & 0xFFFFu);
        v = (uint32_t)i;
    }
    __device__ int plan(RadixState& st, RadixLds&)
    {
        if (threadIdx.x == 0) {
            const bool on = w.status->n_overflow > 0 && w.status->err_range == 0;
            st.active = on ? 1 : 0;
            st.key_min = 0;
            const uint64_t top = (uint64_t)w.width * w.height - 1;
            const int bits = top == 0 ? 0 : 64 - __builtin_clzll(top);
            st.passes = bits <= 8 ? 1 : (bits + 7) / 8;
        }
        return w.status->n_overflow;
    }
    __device__ void store(int64_t, uint64_t, uint32_t) const {}
    __device__ void extra(int q, const uint64_t* keys, const uint32_t* vals, RadixLds&)
    {
        const int tile = w.overflow_tiles[q];
        const int64_t p0 = (int64_t)tile * kLinkTile;
        const int64_t p1 = (p0 + kLinkTile) < w.n ? (p0 + kLinkTile) : w.n;
        const int64_t n = w.n;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += kFbThreads) {
            const uint32_t xy = w.s_xy[p];
            const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
            const uint64_t toa = w.s_toa[p];
            for (int dy = -1; dy <= 1; dy++) {
                const int qy = y + dy;
                if (qy < 0 || qy >= (int)w.height) continue;
                for (int dx = -1; dx <= 1; dx++) {
                    const int qx = x + dx;
                    if (qx < 0 || qx >= (int)w.width) continue;
                    const uint64_t key = (uint64_t)qy * w.width + qx;
                    // [lo, hi): entries of pixel key
                    int64_t a = 0, b = n;
                    while (a < b) {
                        const int64_t m = (a + b) >> 1;
                        if (keys[m] < key) a = m + 1; else b = m;
                    }
                    const int64_t lo = a;
                    b = n;
                    while (a < b) {
                        const int64_t m = (a + b) >> 1;
                        if (keys[m] <= key) a = m + 1; else b = m;
                    }
                    const int64_t hi = a;
                    // last entry with position < p
                    a = lo;
                    b = hi;
                    while (a < b) {
                        const int64_t m = (a + b) >> 1;
                        if ((int64_t)vals[m] < p) a = m + 1; else b = m;
                    }
                    if (a > lo) {
                        const int64_t c = vals[a - 1];
                        if (c < 0 || c >= p) {
                            atomicOr(&w.status->err_internal, 1);
                        } else if (toa - w.s_toa[c] <= w.dt) {
                            gunion(w.gparent, w.s_idx[c], w.s_idx[p], &w.status->err_internal);
                        }
                    }
                }
            }
        }
        signal_done(&w.status->rs[1].query_done);
    }
};

__global__ __launch_bounds__(kFbThreads) void k_link_fallback(Work w)
{
    PixSortJob job{w};
    uint64_t* kb[2] = {w.fb_key[0], w.fb_key[1]};
    uint32_t* vb[2] = {w.fb_val[0], w.fb_val[1]};
    radix_engine(job, &w.status->rs[1], kb, vb, w.fb_hist, w.n_fb_blocks, &w.status->err_internal);
}

int persistent_grid();

hipError_t launch_link_fallback(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_fallback", s);
    hipLaunchKernelGGL(k_link_fallback, dim3(persistent_grid()), dim3(kFbThreads), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------- cross-tile unions
__global__ void k_union_edges(Work w)
{
    if (w.status->err_range) return;
    const int64_t ne = w.status->n_edges < w.edge_cap ? w.status->n_edges : w.edge_cap;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int2 ed = w.edges[e];
        gunion(w.gparent, ed.x, ed.y, &w.status->err_internal);
    }
}

hipError_t launch_union_edges(const Work& w, hipStream_t s)
{
    TimedLaunch tl("union_edges", s);
    hipLaunchKernelGGL(k_union_edges, dim3(256), dim3(256), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------------------ flatten
__global__ void k_flatten(Work w, int32_t* __restrict__ labels)
{
    if (w.status->err_range) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < w.n; i += (int64_t)gridDim.x * blockDim.x)
        labels[i] = gfind(w.gparent, (int32_t)i, &w.status->err_internal);
}

hipError_t launch_flatten(const Work& w, int32_t* labels, hipStream_t s)
{
    TimedLaunch tl("flatten", s);
    int64_t blocks = ((int64_t)w.n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_flatten, dim3((unsigned)blocks), dim3(256), 0, s, w, labels);
    return hipGetLastError();
}

}  // namespace hc
