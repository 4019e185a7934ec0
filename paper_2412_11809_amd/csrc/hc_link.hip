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

// First halo position of every link tile: the earliest sorted position p
// with toa(p) >= toa(p0) - dt (a suffix of the positions before p0, so a
// binary search), or -1 when the halo exceeds kLinkHaloCap or the tile's
// ToA span does not fit 32 bits (such tiles go to the fallback).
__global__ void k_link_halo(Work w)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= w.n_link_tiles || w.status->err_range) return;
    const int64_t p0 = (int64_t)k * kLinkTile;
    const int64_t p1 = (p0 + kLinkTile) < w.n ? (p0 + kLinkTile) : w.n;
    const uint64_t lo = sat_sub_u64(w.s_toa[p0], w.dt);
    const int64_t lim = p0 - kLinkHaloCap > 0 ? p0 - kLinkHaloCap : 0;
    int64_t a = lim, b = p0;
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (w.s_toa[m] < lo) a = m + 1; else b = m;
    }
    bool overflow = (a == lim && lim > 0 && w.s_toa[lim - 1] >= lo);
    overflow |= (w.s_toa[p1 - 1] - w.s_toa[a]) > 0xFFFFFFFFull;
    w.link_h0[k] = overflow ? -1 : (int32_t)a;
}

hipError_t launch_link_halo(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_halo", s);
    hipLaunchKernelGGL(k_link_halo, dim3((w.n_link_tiles + 255) / 256), dim3(256), 0, s, w);
    return hipGetLastError();
}

constexpr uint64_t kEmptySlot = 0ull;

// One work-group per tile of kLinkTile sorted hits (+ halo), all in LDS.
// Dynamic LDS holds an occupancy bitmap of the sensor (bm_words words; 0 =
// no bitmap, every neighbour pixel is looked up in the hash).
__global__ __launch_bounds__(kLinkThreads) void k_link(Work w, int bm_words)
{
    constexpr int LCAP = kLinkTile + kLinkHaloCap;
    constexpr int PER = kLinkTile / kLinkThreads;
    __shared__ uint32_t l_toa[LCAP];
    __shared__ uint32_t l_xy[LCAP];
    __shared__ int32_t l_idx[LCAP];
    __shared__ int32_t l_par[LCAP];
    __shared__ int16_t l_next[LCAP];
    __shared__ unsigned long long h_slot[kLinkHash];  // (pixel key << 32) | list head
    extern __shared__ uint32_t bm[];

    if (w.status->err_range) return;
    const int tile = xcd_tile(w.n_link_tiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)tile * kLinkTile;
    const int64_t p1 = (p0 + kLinkTile) < w.n ? (p0 + kLinkTile) : w.n;
    const int64_t h0 = w.link_h0[tile];
    if (h0 < 0) {  // halo too large: every hit is its own root here, the fallback joins them
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
    const uint32_t W = w.width;
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
    for (int i = t; i < kLinkHash; i += kLinkThreads) h_slot[i] = kEmptySlot;
    for (int i = t; i < bm_words; i += kLinkThreads) bm[i] = 0u;
    __syncthreads();

    // ---- pixel hash (slot per occupied pixel, list of its hits) and bitmap
    for (int i = t; i < L; i += kLinkThreads) {
        const uint32_t xy = l_xy[i];
        const uint32_t key = xy + 1u;
        uint32_t slot = pix_hash(key);
        while (true) {
            const unsigned long long mine = ((unsigned long long)key << 32) | 0xFFFFFFFFull;
            const unsigned long long old = atomicCAS(&h_slot[slot], kEmptySlot, mine);
            if (old == kEmptySlot || (uint32_t)(old >> 32) == key) break;
            slot = (slot + 1u) & (kLinkHash - 1);
        }
        // push onto the slot's list: exchange the low half (the head)
        l_next[i] = (int16_t)atomicExch(reinterpret_cast<int32_t*>(&h_slot[slot]), i);
        if (bm_words) {
            const uint32_t pix = (xy >> 16) * W + (xy & 0xFFFFu);
            atomicOr(&bm[pix >> 5], 1u << (pix & 31u));
        }
    }
    __syncthreads();

    // ---- neighbour search of the tile hits
    const uint64_t dt = w.dt;
    const int H = (int)w.height;
#pragma unroll 1
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        if (i >= L) break;
        const uint32_t xy = l_xy[i];
        const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
        const uint32_t ti = l_toa[i];
        const int xlo = x > 0 ? x - 1 : 0;
        const int xhi = x + 1 < (int)W ? x + 1 : (int)W - 1;
        for (int qy = y - 1; qy <= y + 1; qy++) {
            if (qy < 0 || qy >= H) continue;
            uint32_t occ = (1u << (xhi - xlo + 1)) - 1u;  // bit k: pixel xlo + k
            if (bm_words) {
                const uint32_t pa = (uint32_t)qy * W + (uint32_t)xlo;
                const uint32_t wa = pa >> 5, sh = pa & 31u;
                uint64_t bits = bm[wa];
                if (sh > 29u && wa + 1 < (uint32_t)bm_words) bits |= (uint64_t)bm[wa + 1] << 32;
                occ &= (uint32_t)(bits >> sh);
            }
            while (occ) {
                const int k = __builtin_ctz(occ);
                occ &= occ - 1u;
                const uint32_t key = ((uint32_t)(xlo + k) | ((uint32_t)qy << 16)) + 1u;
                uint32_t slot = pix_hash(key);
                int a = -1;
                while (true) {
                    const unsigned long long v = h_slot[slot];
                    if ((uint32_t)(v >> 32) == key) {
                        a = (int32_t)(uint32_t)v;
                        break;
                    }
                    if (v == kEmptySlot) break;
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
    const uint64_t pixels = (uint64_t)w.width * w.height;
    const int bm_words = pixels <= (uint64_t)kLinkBitmapMaxWords * 32 ? (int)((pixels + 31) / 32) : 0;
    hipLaunchKernelGGL(k_link, dim3(xcd_grid(w.n_link_tiles)), dim3(kLinkThreads), (size_t)bm_words * 4, s, w,
                       bm_words);
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
    if (!w.status->n_overflow || w.status->err_range) return;  // the common case
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
// labels[i] = root(i).  One work-group per block of kScanBlock indices; a
// root (labels[i] == i) is a cluster: its bit is set in the block's mask and
// the block's root count is stored for the compaction scan.
__global__ __launch_bounds__(kScanThreads) void k_flatten(Work w, int32_t* __restrict__ labels)
{
    static_assert(kScanBlock == 8 * kScanThreads && kScanThreads % kWave == 0, "mask layout");
    __shared__ uint32_t wsum[kScanThreads / kWave];
    if (w.status->err_range) return;
    const int b = blockIdx.x;
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    const int64_t base = (int64_t)b * kScanBlock;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kScanBlock / kScanThreads; q++) {
        const int64_t i = base + q * kScanThreads + t;
        bool root = false;
        if (i < w.n) {
            const int32_t r = gfind(w.gparent, (int32_t)i, &w.status->err_internal);
            labels[i] = r;
            root = (r == (int32_t)i);
        }
        const unsigned long long m = __ballot(root);
        if (lane == 0) w.root_mask[(int64_t)b * (kScanBlock / 64) + q * (kScanThreads / kWave) + wid] = m;
        c += root;
    }
    uint32_t total;
    block_exclusive_scan<kScanThreads>(c, wsum, &total);
    if (t == 0) w.blk_count[b] = total;
}

hipError_t launch_flatten(const Work& w, int32_t* labels, hipStream_t s)
{
    TimedLaunch tl("flatten", s);
    hipLaunchKernelGGL(k_flatten, dim3(w.n_scan_blocks), dim3(kScanThreads), 0, s, w, labels);
    return hipGetLastError();
}

}  // namespace hc
