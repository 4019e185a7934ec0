// Steps A2 and A3 of the clustering path: neighbour search and union-find.
//
// The paper (Section 4.1) sweeps the ToA-sorted hits, finds for each hit the
// latest earlier hit at its own pixel and at each of its eight neighbours
// through a per-pixel matrix, and joins the clusters with union-find.
// Its GPU version gives every thread one chunk and one full 256 x 256 matrix.
//
// Here each work-group takes a tile of kLinkTile consecutive sorted hits plus
// the "halo" of earlier hits whose ToA lies within dt of the tile's first hit,
// and works entirely in LDS:
//   * an occupancy bitmap of the sensor and the popcount prefix of its words
//     give every occupied pixel of the tile a dense rank, and a CSR lists the
//     tile's hits per pixel rank -- the tile-sized replacement of the paper's
//     dense matrix;
//   * each tile hit joins, at each of its 9 pixels, an earlier hit within dt
//     (the paper's matrix holds the latest one; any gives the same clusters,
//     see k_link);
//   * the joins are applied in bulk rounds in an LDS forest whose roots are
//     the earliest slots (the paper's time-ordered roots); the smallest input
//     index of every tree is the label candidate written to the global parent
//     array, and halo hits joined by the tile are queued as cross-tile edges.
// Sensors too large for the bitmap (or a caller's flag) use k_link_window,
// which scans each hit's dt window instead.  A tile whose halo does not fit
// goes to k_link_wide, the same index over the tile and a halo of up to 7168
// hits in one large work-group; a tile whose halo exceeds even that (or whose
// ToA span exceeds 32 bits) is handled by k_link_fallback: a pixel-sorted copy
// of the hits in such tiles' windows plus binary searches.  k_union_edges applies
// the queued cross-tile edges with atomic compare-and-swap, and k_flatten
// writes labels[i] = root(i).
#include "hc_device.h"
#include "hc_radix.h"

namespace hc {

// Which neighbour search runs: the pixel index (k_link) whenever the
// sensor's occupancy bitmap fits in LDS, else the window scan (k_link_window,
// coordinates below 2^14); a caller's flag can force either.  The index is
// faster on every stream measured, sparse or dense, so it is the default.
enum { kLinkWindow = 0, kLinkIndex = 1 };
__host__ __device__ inline int link_kernel(const Work& w)
{
    const bool win_ok = w.width <= kLinkWindowMaxDim && w.height <= kLinkWindowMaxDim;
    const bool idx_ok = (uint64_t)w.width * w.height <= kLinkMaxPixels;
    if (w.link_mode == 1 || !win_ok) return kLinkIndex;
    if (w.link_mode == 2 || !idx_ok) return kLinkWindow;
    return kLinkIndex;
}

// First halo position of every link tile: the earliest sorted position p
// with toa(p) >= toa(p0) - dt (a suffix of the positions before p0, so a
// binary search), or -1 when the halo exceeds kLinkHaloCap, the tile's ToA
// span does not fit 32 bits or the sensor is too large for the LDS pixel
// bitmap (such tiles go to the fallback).
__global__ void k_link_halo(Work w)
{
    resolve_count(w);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= w.n_link_tiles || w.status->err_range) return;
    const TileRange tr = tile_range(w, kLinkKind, k, kLinkTile);
    const int64_t p0 = tr.start;
    const int64_t p1 = tr.start + tr.count;
    const uint64_t lo = sat_sub_u64(w.s_toa[p0], seg_dt(w, tr.seg));
    // the halo never reaches into the previous chunk
    const int64_t lim = p0 - kLinkHaloCap > tr.seg_start ? p0 - kLinkHaloCap : tr.seg_start;
    int64_t a = lim, b = p0;
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (w.s_toa[m] < lo) a = m + 1; else b = m;
    }
    bool overflow = (a == lim && lim > tr.seg_start && w.s_toa[lim - 1] >= lo);
    overflow |= (w.s_toa[p1 - 1] - w.s_toa[a]) > 0xFFFFFFFFull;
    overflow |= link_kernel(w) == kLinkIndex && (uint64_t)w.width * w.height > kLinkMaxPixels;  // no bitmap room
    w.link_h0[k] = overflow ? -1 : (int32_t)a;
}

hipError_t launch_link_halo(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_halo", s);
    hipLaunchKernelGGL(k_link_halo, dim3((w.n_link_tiles + 255) / 256), dim3(256), 0, s, w);
    return hipGetLastError();
}

// Global loads of a link tile, ordered so that the halo start is the only
// thing that waits on a round trip: the error flag, the halo start and the
// tile's own hits (whose positions are known) are requested together; the
// halo hits and the ToA base follow.  Thread t holds the tile hits at slots
// hl + t + q * kLinkThreads (q < PER) and the halo hits at slots
// t + q * kLinkThreads below hl (q < 2).  Returns false when the work-group
// has to stop: the error flag is set, or the halo does not fit, in which case
// the tile's hits become their own roots and the tile goes to the fallback.
template <int PER>
__device__ inline bool link_tile_load(const Work& w, int tile, const TileRange& tr, int64_t& h0, uint64_t& tbase,
                                      uint64_t (&ttoa)[PER], uint32_t (&txy)[PER], int32_t (&tid)[PER],
                                      uint64_t (&htoa)[2], uint32_t (&hxy)[2], int32_t (&hid)[2])
{
    const int t = threadIdx.x;
    const int64_t p0 = tr.start;
    const int64_t p1 = tr.start + tr.count;
    const int err = w.status->err_range;
    h0 = w.link_h0[tile];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t p = p0 + t + q * kLinkThreads;
        tid[q] = -1;
        if (p < p1) {
            ttoa[q] = w.s_toa[p];
            txy[q] = w.s_xy[p];
            tid[q] = w.s_idx[p];
        }
    }
    if (err) return false;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t p = p0 + t + q * kLinkThreads;
        if (p < p1 && (tid[q] < 0 || tid[q] >= w.n)) {
            atomicOr(&w.status->err_internal, 1);
            tid[q] = 0;
        }
    }
    if (h0 < 0) {  // halo too large: every hit is its own root here, the fallback joins them
#pragma unroll
        for (int q = 0; q < PER; q++)
            if (p0 + t + q * kLinkThreads < p1) w.gparent[tid[q]] = tid[q];
        if (t == 0) {
            const int k = atomicAdd(&w.status->n_overflow, 1);
            w.overflow_tiles[k] = tile;
            w.tile_nedge[tile] = 0;
        }
        return false;
    }
    const int hl = (int)(p0 - h0);
    tbase = w.s_toa[h0];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int a = t + q * kLinkThreads;
        hid[q] = -1;
        if (a < hl) {
            const int64_t p = h0 + a;
            htoa[q] = w.s_toa[p];
            hxy[q] = w.s_xy[p];
            int32_t id = w.s_idx[p];
            if (id < 0 || id >= w.n) {
                atomicOr(&w.status->err_internal, 1);
                id = 0;
            }
            hid[q] = id;
        }
    }
    return true;
}

// Joins of one tile (cand: per tile hit, the slot joined at each of its 9
// pixels, or -1) applied in the LDS forest l_par: first every tile hit hangs
// under its smallest candidate (a plain store by its own thread) and every
// slot walks to its root; then bulk rounds hook every edge's larger root
// under the smaller (atomic minimum) and retire the edges already inside one
// tree, then walk every slot to its root; repeat until no edge joins two
// roots.  Then the
// smallest input index of every local tree is published: as the parent of
// the tree's tile hits, and as cross-tile edges for its halo hits.
// minidx: LDS scratch of L words (the caller's ToA array, no longer read).
template <int PER>
__device__ inline void link_union_publish(const Work& w, int tile, int32_t* l_par, int (&cand)[PER][9],
                                          const int32_t (&tid)[PER], const int32_t (&hid)[2], int hl, int L,
                                          int32_t* minidx)
{
    const int t = threadIdx.x;
    // first round without atomics: every tile hit hangs under its smallest
    // candidate (only its own thread writes its pointer), then the walks
    __syncthreads();  // the caller's search has read the slots' data
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        if (i >= L) continue;
        int mn = i;
#pragma unroll
        for (int k = 0; k < 9; k++)
            if (cand[q][k] >= 0 && cand[q][k] < mn) mn = cand[q][k];
        l_par[i] = mn;
    }
    __syncthreads();
    for (int x = t; x < L; x += kLinkThreads) {
        int p = l_par[x];
        while (true) {
            const int g = l_par[p];
            if (g == p) break;
            l_par[x] = g;
            p = g;
        }
    }
    __syncthreads();
    while (true) {
        bool changed = false;
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int i = hl + t + q * kLinkThreads;
            // the AND of the candidates is negative only when all are (retired)
            int live = cand[q][0];
#pragma unroll
            for (int k = 1; k < 9; k++) live &= cand[q][k];
            if (i >= L || live < 0) continue;
            const int pi = l_par[i];
#pragma unroll
            for (int k = 0; k < 9; k++) {
                if (cand[q][k] < 0) continue;
                const int pc = l_par[cand[q][k]];
                if (pc != pi) {
                    atomicMin(&l_par[pc > pi ? pc : pi], pc > pi ? pi : pc);
                    changed = true;
                } else {
                    // joined: retire the edge.  The pointers just read may be
                    // hooks of this round that a smaller atomic minimum later
                    // replaces, but the edge that made each such hook saw
                    // different roots, so it stays and is checked again next
                    // round; a round without hooks reads only settled trees.
                    cand[q][k] = -1;
                }
            }
        }
        // a round without hooks leaves the forest as the last walk left it:
        // every pointer already names its root
        if (!__syncthreads_or(changed)) break;
        // every slot walks to its root, shortening its own pointer at each
        // step: the walks of later slots on the same path reuse those jumps
        // (a pointer only ever moves to an ancestor, so any value read is valid)
        for (int x = t; x < L; x += kLinkThreads) {
            int p = l_par[x];
            while (true) {
                const int g = l_par[p];
                if (g == p) break;
                l_par[x] = g;
                p = g;
            }
        }
        __syncthreads();
    }

    // ---- smallest input index per local tree, then publish
    for (int i = t; i < L; i += kLinkThreads) minidx[i] = 0x7FFFFFFF;
    __syncthreads();
    int32_t rt[PER], rh[2];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        rt[q] = i < L ? l_par[i] : -1;
        if (rt[q] >= 0) atomicMin(&minidx[rt[q]], tid[q]);
    }
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int a = t + q * kLinkThreads;
        rh[q] = a < hl ? l_par[a] : -1;
        if (rh[q] >= 0) atomicMin(&minidx[rh[q]], hid[q]);
    }
    __syncthreads();
    // halo hits joined by this tile become cross-tile edges, in the tile's
    // own region of kLinkHaloCap entries (positions from a block scan)
    int32_t mh[2];
    uint32_t ne = 0;
#pragma unroll
    for (int q = 0; q < 2; q++) {
        mh[q] = rh[q] >= 0 ? minidx[rh[q]] : -1;
        ne += (rh[q] >= 0 && hid[q] != mh[q]) ? 1u : 0u;
    }
    __shared__ uint32_t e_wsum[kLinkThreads / kWave];
    uint32_t n_tile_edges;
    uint32_t pos = block_exclusive_scan<kLinkThreads>(ne, e_wsum, &n_tile_edges);
    if (t == 0) w.tile_nedge[tile] = (int32_t)n_tile_edges;
    const int64_t e_base = (int64_t)tile * kLinkHaloCap;
#pragma unroll
    for (int q = 0; q < PER; q++)
        if (rt[q] >= 0) w.gparent[tid[q]] = minidx[rt[q]];
#pragma unroll
    for (int q = 0; q < 2; q++)
        if (rh[q] >= 0 && hid[q] != mh[q])
            w.edges[e_base + pos++] = make_int2(hid[q], mh[q]);  // pos < hl <= kLinkHaloCap
}

// Window scan of the tile hits (see k_link_window): for tile hit i, the
// earlier slots [lo[q], i) hold every earlier hit within dt; walking them
// backwards, the first hit met at each of the 9 pixels is the latest there.
// l_xy: packed (y << 16 | x), both below 2^14.
template <int PER>
__device__ inline void link_window_search(const uint32_t* l_toa, const uint32_t* l_xy, int hl, int L,
                                          const int (&lo)[PER], int (&cand)[PER][9])
{
    constexpr uint32_t kGuard = 0x40004000u, kMask = 0xFFFCFFFCu;
    const int t = threadIdx.x;
    (void)l_toa;
#pragma unroll
    for (int q = 0; q < PER; q++) {
#pragma unroll
        for (int k = 0; k < 9; k++) cand[q][k] = -1;
        const int i = hl + t + q * kLinkThreads;
        if (i >= L) continue;
        const uint32_t c = l_xy[i] - 0x00010001u;
        uint32_t found = 0;
        for (int j = i - 1; j >= lo[q]; j--) {
            const uint32_t r = (l_xy[j] | kGuard) - c;
            if ((r & kMask) == kGuard) {
                const uint32_t ax = r & 3u, ay = (r >> 16) & 3u;
                if (ax == 3u || ay == 3u) continue;
                const int dir = (int)(ay * 3u + ax);
                if ((found >> dir) & 1u) continue;
                found |= 1u << dir;
#pragma unroll
                for (int k = 0; k < 9; k++)
                    if (k == dir) cand[q][k] = j;
                if (found == 0x1FFu) break;
            }
        }
    }
}

// x, y of a pixel id p = y * W + x.  16-bit ids (sensors of at most 2^16
// pixels) divide by multiplying with magic = ceil(2^32 / W), exact for every
// p < 2^16 because the rounding error of magic times p stays below 2^32.
template <typename PixT>
__device__ inline void pix_xy(uint32_t p, uint32_t W, uint32_t magic, int& x, int& y)
{
    const uint32_t q = sizeof(PixT) == 2 ? (W > 1 ? __umulhi(p, magic) : p) : p / W;
    y = (int)q;
    x = (int)(p - q * W);
}

// Dense rank (in pixel order) of an occupied pixel: set bits before it in the
// occupancy bitmap, from the 16-bit prefix count of its 64-bit word.
__device__ inline uint32_t pix_rank(uint32_t p, const uint64_t* bm, const uint16_t* wpre)
{
    const uint32_t wd = p >> 6;
    return wpre[wd] + (uint32_t)__popcll(bm[wd] & ((1ull << (p & 63u)) - 1ull));
}

// Count one slot at its pixel: its rank, and its place among the slots of
// that pixel (the 16-bit count it saw; two counters share a word, and counts
// stay below 2^16, so no carry crosses halves).
__device__ inline uint32_t pix_count(uint32_t p, const uint64_t* bm, const uint16_t* wpre, uint32_t* pcount)
{
    const uint32_t r = pix_rank(p, bm, wpre);
    const uint32_t half = 16u * (r & 1u);
    return r | (((atomicAdd(&pcount[r >> 1], 1u << half) >> half) & 0xFFFFu) << 16);
}

// One work-group per tile of kLinkTile sorted hits (+ halo), all in LDS.
//
// Local slots 0..L-1 are the sorted positions h0..p1-1, so a smaller slot is
// an earlier hit.  A tile-sized index of the occupied pixels replaces the
// paper's per-pixel "last hit" matrix:
//   * an occupancy bitmap of the sensor plus the popcount prefix of its 64-bit
//     words gives every occupied pixel a dense rank (pixel order);
//   * a CSR lists, per occupied pixel, the slots of its hits (in no particular
//     order), so the three pixels of a neighbour row are three consecutive
//     segments.
// The matrix would join a hit to the LATEST earlier hit at each neighbour
// pixel (within dt).  Joining it to ANY earlier hit there within dt gives the
// same clusters: the hits of one pixel whose ToAs lie within one dt of each
// other are always connected among themselves (each joins an earlier one
// within dt, by induction over time), and the latest earlier hit and the one
// chosen both lie in the dt before the joining hit.  So the index needs no
// order inside a pixel's list: the first entry of the segment that is earlier
// and within dt is taken (usually the only entry).
// link_union_publish then applies the joins and publishes the labels.
// Hits are kept as pixel ids (16-bit up to 2^16 pixels): with the 64-bit
// word prefixes the tile's LDS stays below 40 KiB on a 256 x 256 sensor, so
// four work-groups share a CU (the kernel is latency bound: occupancy is what
// speeds it up).  Dynamic LDS: the bitmap (bm64 words), then the prefixes.
template <typename PixT>
__global__ __launch_bounds__(kLinkThreads, 8) void k_link(Work w, int bm64, uint32_t magic)
{
    resolve_count(w);
    constexpr int LCAP = kLinkTile + kLinkHaloCap;
    constexpr int PER = kLinkTile / kLinkThreads;
    constexpr int LPER = LCAP / kLinkThreads;
    __shared__ uint32_t l_toa[LCAP];      // ToA - tile base; then minima
    __shared__ PixT l_pix[LCAP];          // pixel id y * W + x
    __shared__ int32_t l_par[LCAP];
    __shared__ uint16_t csr[LCAP];        // slots grouped by pixel rank
    __shared__ uint16_t pstart[LCAP + 2]; // counts (packed in pairs), then start of each rank's CSR segment
    __shared__ uint32_t wsum[kLinkThreads / kWave];
    extern __shared__ uint64_t dyn64[];
    uint64_t* bm = dyn64;
    uint32_t* bm32 = reinterpret_cast<uint32_t*>(dyn64);
    uint16_t* wpre = reinterpret_cast<uint16_t*>(dyn64 + bm64);
    uint32_t* pcount = reinterpret_cast<uint32_t*>(pstart);  // two 16-bit counters per word

    const int tile = xcd_tile(w.n_link_tiles, w.xcd_map);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
    int64_t h0;
    uint64_t tbase, ttoa[PER], htoa[2];
    uint32_t txy[PER], hxy[2];
    int32_t tid[PER], hid[2];
    if (!link_tile_load<PER>(w, tile, tr, h0, tbase, ttoa, txy, tid, htoa, hxy, hid)) return;
    const int64_t p1 = tr.start + tr.count;
    const int L = (int)(p1 - h0);
    const int hl = (int)(tr.start - h0);
    const uint32_t W = w.width;
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int a = t + q * kLinkThreads;
        if (a < hl) {
            l_toa[a] = (uint32_t)(htoa[q] - tbase);
            l_pix[a] = (PixT)((hxy[q] >> 16) * W + (hxy[q] & 0xFFFFu));
            l_par[a] = a;
        }
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        if (i < L) {
            l_toa[i] = (uint32_t)(ttoa[q] - tbase);
            l_pix[i] = (PixT)((txy[q] >> 16) * W + (txy[q] & 0xFFFFu));
            l_par[i] = i;
        }
    }
    __syncthreads();

    const uint64_t dt = seg_dt(w, tr.seg);
    int cand[PER][9];
    {
        for (int i = t; i < bm64; i += kLinkThreads) bm[i] = 0ull;
        for (int i = t; i < (LCAP + 2) / 2; i += kLinkThreads) pcount[i] = 0u;
        __syncthreads();
        // ---- occupancy bitmap
        for (int i = t; i < L; i += kLinkThreads) {
            const uint32_t p = l_pix[i];
            atomicOr(&bm32[p >> 5], 1u << (p & 31u));
        }
        __syncthreads();
        // ---- popcount prefix of the 64-bit bitmap words
        {
            const int per = (bm64 + kLinkThreads - 1) / kLinkThreads;
            const int w0 = t * per;
            uint32_t c = 0;
            for (int k = 0; k < per; k++)
                if (w0 + k < bm64) c += (uint32_t)__popcll(bm[w0 + k]);
            uint32_t run = block_exclusive_scan<kLinkThreads>(c, wsum, nullptr);
            for (int k = 0; k < per; k++)
                if (w0 + k < bm64) {
                    wpre[w0 + k] = (uint16_t)run;
                    run += (uint32_t)__popcll(bm[w0 + k]);
                }
        }
        __syncthreads();
        // ---- hits per occupied pixel (counts stay below 2^16: no carry between
        // halves); the count a hit sees is its place in its pixel's segment
        uint32_t rp[LPER];  // pixel rank | place in the segment << 16
#pragma unroll
        for (int q = 0; q < LPER; q++) {
            const int i = t + q * kLinkThreads;
            if (i < L) {
                const uint32_t r = pix_rank(l_pix[i], bm, wpre);
                const uint32_t half = 16u * (r & 1u);
                rp[q] = r | (((atomicAdd(&pcount[r >> 1], 1u << half) >> half) & 0xFFFFu) << 16);
            }
        }
        __syncthreads();
        // ---- exclusive scan of the counts -> first CSR position per pixel rank
        {
            uint32_t c[LPER];
            uint32_t sum = 0;
#pragma unroll
            for (int k = 0; k < LPER; k++) {
                c[k] = pstart[t * LPER + k];
                sum += c[k];
            }
            uint32_t run = block_exclusive_scan<kLinkThreads>(sum, wsum, nullptr);
#pragma unroll
            for (int k = 0; k < LPER; k++) {
                pstart[t * LPER + k] = (uint16_t)run;
                run += c[k];
            }
            if (t == kLinkThreads - 1) pstart[LCAP] = (uint16_t)run;  // end of the last segment
        }
        __syncthreads();
        // ---- fill: segment r is [pstart[r], pstart[r + 1])
#pragma unroll
        for (int q = 0; q < LPER; q++) {
            const int i = t + q * kLinkThreads;
            if (i < L) csr[pstart[rp[q] & 0xFFFFu] + (rp[q] >> 16)] = (uint16_t)i;
        }
        __syncthreads();
        // ---- neighbour search: an earlier hit within dt per neighbour pixel.
        // Branch-free stages, so the LDS reads of all 9 pixels overlap: the
        // three rows' bitmap bits and first ranks, the 9 segment bounds, the
        // segments' first entries, their ToAs.  Empty pixels read slot 0 and
        // discard it.  Only a segment whose first entry does not qualify
        // (a pixel hit more than once in the tile) is walked further.
        const int H = (int)w.height;
        const uint32_t dt32 = dt < 0xFFFFFFFFull ? (uint32_t)dt : 0xFFFFFFFFu;
#pragma unroll
        for (int q = 0; q < PER; q++) {
#pragma unroll
            for (int k = 0; k < 9; k++) cand[q][k] = -1;
            const int i = hl + t + q * kLinkThreads;
            if (i >= L) continue;
            int x, y;
            pix_xy<PixT>(l_pix[i], W, magic, x, y);
            const uint32_t ti = l_toa[i];
            const int xlo = x > 0 ? x - 1 : 0;
            const int xhi = x + 1 < (int)W ? x + 1 : (int)W - 1;
            const uint32_t rowmask = (1u << (xhi - xlo + 1)) - 1u;
            uint32_t occ[3];
            int rk0[3];
#pragma unroll
            for (int rr = 0; rr < 3; rr++) {
                const int qy = y - 1 + rr;
                const bool rowok = qy >= 0 && qy < H;
                const uint32_t pa = rowok ? (uint32_t)qy * W + (uint32_t)xlo : 0u;
                const uint32_t wa = pa >> 6, sh = pa & 63u;
                const uint64_t b0 = bm[wa];
                const uint64_t b1 = bm[(int)wa + 1 < bm64 ? wa + 1 : wa];
                uint64_t bits = b0 >> sh;
                if (sh > 61u) bits |= b1 << (64u - sh);
                occ[rr] = rowok ? (uint32_t)bits & rowmask : 0u;
                rk0[rr] = (int)(wpre[wa] + (uint32_t)__popcll(b0 & ((1ull << sh) - 1ull)));
            }
            int s0[9], s1[9];
#pragma unroll
            for (int d = 0; d < 9; d++) {
                const uint32_t o = occ[d / 3];
                const bool has = (o >> (d % 3)) & 1u;
                const int r = has ? rk0[d / 3] + __popc(o & ((1u << (d % 3)) - 1u)) : 0;
                const int b = pstart[r];
                const int e = pstart[r + 1];
                s0[d] = has ? b : 0;
                s1[d] = has ? e : 0;
            }
            int v[9];
#pragma unroll
            for (int d = 0; d < 9; d++) v[d] = csr[s0[d] < s1[d] ? s0[d] : 0];
#pragma unroll
            for (int d = 0; d < 9; d++) {
                const uint32_t tv = l_toa[v[d]];
                if (s0[d] < s1[d] && v[d] < i && ti - tv <= dt32) {
                    cand[q][d] = v[d];
                } else if (s1[d] - s0[d] > 1) {
                    for (int j = s0[d] + 1; j < s1[d]; j++) {
                        const int u = csr[j];
                        if (u < i && ti - l_toa[u] <= dt32) {
                            cand[q][d] = u;
                            break;
                        }
                    }
                }
            }
        }
    }
    link_union_publish(w, tile, l_par, cand, tid, hid, hl, L, reinterpret_cast<int32_t*>(l_toa));
}

// Same contract as k_link, without a pixel index: the latest earlier hit at
// each neighbour pixel is found by scanning the tile's time window backwards.
// Every earlier hit within dt of hit i sits in the slots [lo_i, i), because
// the slots are in (ToA, index) order; walking them from i - 1 down, the first
// hit met at each of the 9 pixels is the latest one there.  The spatial test
// is two 16-bit lanes in one 32-bit word: with x and y below 2^14 and guard
// bit 14 set in both lanes of the earlier hit's word, the difference
// g_j - (e_i - 0x10001) holds 0x4000 + dx + 1 per lane with no borrow between
// lanes, so (diff & 0xFFFCFFFC) == 0x40004000 keeps dx, dy in -1..2; dx or dy
// of 2 (low bits 3) is rejected inside the rarely taken branch.
// Sparse input gives short windows (a few slots); inside a dense shower the
// window holds every hit of the last dt.
__global__ __launch_bounds__(kLinkThreads, 8) void k_link_window(Work w)
{
    resolve_count(w);
    constexpr int LCAP = kLinkTile + kLinkHaloCap;
    constexpr int PER = kLinkTile / kLinkThreads;
    __shared__ uint32_t l_toa[LCAP];
    __shared__ uint32_t l_xy[LCAP];
    __shared__ int32_t l_par[LCAP];

    const int tile = xcd_tile(w.n_link_tiles, w.xcd_map);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
    int64_t h0;
    uint64_t tbase, ttoa[PER], htoa[2];
    uint32_t txy[PER], hxy[2];
    int32_t tid[PER], hid[2];
    if (!link_tile_load<PER>(w, tile, tr, h0, tbase, ttoa, txy, tid, htoa, hxy, hid)) return;
    const int64_t p1 = tr.start + tr.count;
    const int L = (int)(p1 - h0);
    const int hl = (int)(tr.start - h0);
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int a = t + q * kLinkThreads;
        if (a < hl) {
            l_toa[a] = (uint32_t)(htoa[q] - tbase);
            l_xy[a] = hxy[q];
            l_par[a] = a;
        }
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        if (i < L) {
            l_toa[i] = (uint32_t)(ttoa[q] - tbase);
            l_xy[i] = txy[q];
            l_par[i] = i;
        }
    }
    __syncthreads();

    const uint64_t dt = seg_dt(w, tr.seg);
    int lo[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        lo[q] = i;
        if (i >= L) continue;
        const uint32_t ti = l_toa[i];
        int a = 0;
        if (dt < (uint64_t)ti) {  // first slot with toa >= ti - dt (ToAs ascend with the slot)
            const uint32_t th = ti - (uint32_t)dt;
            int b = i;
            while (a < b) {
                const int m = (a + b) >> 1;
                if (l_toa[m] < th) a = m + 1; else b = m;
            }
        }
        lo[q] = a;
    }
    int cand[PER][9];
    link_window_search<PER>(l_toa, l_xy, hl, L, lo, cand);
    link_union_publish(w, tile, l_par, cand, tid, hid, hl, L, reinterpret_cast<int32_t*>(l_toa));
}

// The pixel-index kernel, or the window-scan kernel.
hipError_t launch_link(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link", s);
    const dim3 grid(xcd_grid(w.n_link_tiles));
    if (link_kernel(w) == kLinkWindow) {
        hipLaunchKernelGGL(k_link_window, grid, dim3(kLinkThreads), 0, s, w);
    } else {
        const uint64_t pixels = (uint64_t)w.width * w.height;
        const int bm64 = (int)((pixels + 63) / 64);
        const size_t dyn = (size_t)bm64 * 8 + (((size_t)bm64 * 2 + 7) & ~(size_t)7);
        const uint32_t magic = w.width > 1 ? (uint32_t)(((1ull << 32) + w.width - 1) / w.width) : 0u;
        if (pixels <= 65536u)
            hipLaunchKernelGGL(k_link<uint16_t>, grid, dim3(kLinkThreads), dyn, s, w, bm64, magic);
        else
            hipLaunchKernelGGL(k_link<uint32_t>, grid, dim3(kLinkThreads), dyn, s, w, bm64, magic);
    }
    return hipGetLastError();
}

// ------------------------------------ wide tiles (halo above kLinkHaloCap)
// Second level for the tiles whose halo did not fit k_link (more than
// kLinkHaloCap hits within dt before the tile, as inside a dense shower):
// one 1024-thread work-group per tile builds the same pixel index (bitmap,
// prefixes, CSR of (ToA, slot, x mod 4) runs) over the tile and a halo of up
// to kWideCap - kLinkTile hits, searches the three neighbour rows of every
// tile hit, joins the candidates in an LDS forest as k_link does, and then
// joins every slot to the smallest input index of its local tree through the
// global union-find (k_link left the tile's hits as their own roots).  Every
// change to the global forest in this launch is a compare-and-swap union, so
// tiles processed together never undo each other's joins, and each targets
// its own slot's root rather than one shared root.  Work is proportional to
// the tile and its halo.
// Tiles whose halo exceeds even this, or whose ToA span does not fit 32 bits,
// or whose sensor has no room for the bitmap, go on to k_link_fallback.
constexpr int kWideThreads = 1024;
constexpr int kWideCap = 8192;
constexpr int kWidePer = kWideCap / kWideThreads;

__global__ __launch_bounds__(kWideThreads) void k_link_wide(Work w, int bm64)
{
    resolve_count(w);
    if (!w.status->n_overflow || w.status->err_range) return;  // the common case
    __shared__ uint2 csr[kWideCap];            // CSR of (ToA - base, slot | (x & 3) << 16); then minima
    __shared__ int32_t l_par[kWideCap];
    __shared__ uint16_t pstart[kWideCap + 2];
    __shared__ uint32_t wsum[kWideThreads / kWave];
    __shared__ int64_t s_h0;
    extern __shared__ uint64_t dyn64[];
    uint64_t* bm = dyn64;
    uint32_t* bm32 = reinterpret_cast<uint32_t*>(dyn64);
    uint16_t* wpre = reinterpret_cast<uint16_t*>(dyn64 + bm64);
    uint32_t* pcount = reinterpret_cast<uint32_t*>(pstart);
    int32_t* minidx = reinterpret_cast<int32_t*>(csr);
    const int t = threadIdx.x;
    const int n_over = w.status->n_overflow;
    const uint32_t W = w.width;
    const int H = (int)w.height;
    for (int q = blockIdx.x; q < n_over; q += gridDim.x) {
        const int tile = w.overflow_tiles[q];
        const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
        const int64_t p0 = tr.start;
        const int64_t p1 = tr.start + tr.count;
        const uint64_t dt = seg_dt(w, tr.seg);
        if (t == 0) {
            const uint64_t lo = sat_sub_u64(w.s_toa[p0], dt);
            const int64_t lim = p0 - (kWideCap - kLinkTile) > tr.seg_start ? p0 - (kWideCap - kLinkTile) : tr.seg_start;
            int64_t a = lim, b = p0;
            while (a < b) {
                const int64_t m = (a + b) >> 1;
                if (w.s_toa[m] < lo) a = m + 1; else b = m;
            }
            bool deep = bm64 == 0 || (a == lim && lim > tr.seg_start && w.s_toa[lim - 1] >= lo);
            deep |= (w.s_toa[p1 - 1] - w.s_toa[a]) > 0xFFFFFFFFull;
            if (deep) w.deep_tiles[atomicAdd(&w.status->n_deep, 1)] = tile;
            s_h0 = deep ? -1 : a;
        }
        for (int i = t; i < bm64; i += kWideThreads) bm[i] = 0ull;
        for (int i = t; i < (kWideCap + 2) / 2; i += kWideThreads) pcount[i] = 0u;
        __syncthreads();
        const int64_t h0 = s_h0;
        if (h0 >= 0) {
            const int L = (int)(p1 - h0);
            const int hl = (int)(p0 - h0);
            const uint64_t tbase = w.s_toa[h0];
            // this thread's slots t + k * kWideThreads (tile and halo alike)
            uint32_t rel[kWidePer], sxy[kWidePer], sp[kWidePer], srp[kWidePer];
            int32_t sid[kWidePer];
#pragma unroll
            for (int k = 0; k < kWidePer; k++) {
                const int a = t + k * kWideThreads;
                sid[k] = -1;
                if (a < L) {
                    rel[k] = (uint32_t)(w.s_toa[h0 + a] - tbase);
                    sxy[k] = w.s_xy[h0 + a];
                    sid[k] = w.s_idx[h0 + a];
                    if (sid[k] < 0 || sid[k] >= w.n) {
                        atomicOr(&w.status->err_internal, 1);
                        sid[k] = 0;
                    }
                    sp[k] = (sxy[k] >> 16) * W + (sxy[k] & 0xFFFFu);
                    atomicOr(&bm32[sp[k] >> 5], 1u << (sp[k] & 31u));
                }
            }
            __syncthreads();
            {
                const int per = (bm64 + kWideThreads - 1) / kWideThreads;
                const int w0 = t * per;
                uint32_t c = 0;
                for (int k = 0; k < per; k++)
                    if (w0 + k < bm64) c += (uint32_t)__popcll(bm[w0 + k]);
                uint32_t run = block_exclusive_scan<kWideThreads>(c, wsum, nullptr);
                for (int k = 0; k < per; k++)
                    if (w0 + k < bm64) {
                        wpre[w0 + k] = (uint16_t)run;
                        run += (uint32_t)__popcll(bm[w0 + k]);
                    }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kWidePer; k++)
                if (t + k * kWideThreads < L) srp[k] = pix_count(sp[k], bm, wpre, pcount);
            __syncthreads();
            {
                uint32_t c[kWidePer];
                uint32_t sum = 0;
#pragma unroll
                for (int k = 0; k < kWidePer; k++) {
                    c[k] = pstart[t * kWidePer + k];
                    sum += c[k];
                }
                uint32_t run = block_exclusive_scan<kWideThreads>(sum, wsum, nullptr);
#pragma unroll
                for (int k = 0; k < kWidePer; k++) {
                    pstart[t * kWidePer + k] = (uint16_t)run;
                    run += c[k];
                }
                if (t == kWideThreads - 1) pstart[kWideCap] = (uint16_t)run;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kWidePer; k++) {
                const int a = t + k * kWideThreads;
                if (a < L) {
                    csr[pstart[srp[k] & 0xFFFFu] + (srp[k] >> 16)] =
                        make_uint2(rel[k], (uint32_t)a | ((sxy[k] & 3u) << 16));
                    l_par[a] = a;
                }
            }
            __syncthreads();
            // ---- candidates of tile hit t (slot hl + t): the first earlier
            // entry within dt at each of its 9 pixels
            const uint32_t dt32 = dt < 0xFFFFFFFFull ? (uint32_t)dt : 0xFFFFFFFFu;
            int cand[9];
#pragma unroll
            for (int k = 0; k < 9; k++) cand[k] = -1;
            const int i = hl + t;
            if (t < tr.count) {
                const uint32_t xy = w.s_xy[p0 + t];
                const uint32_t ti = (uint32_t)(w.s_toa[p0 + t] - tbase);
                const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
                const int xlo = x > 0 ? x - 1 : 0;
                const int xhi = x + 1 < (int)W ? x + 1 : (int)W - 1;
                const uint32_t rowmask = (1u << (xhi - xlo + 1)) - 1u;
#pragma unroll
                for (int rr = 0; rr < 3; rr++) {
                    const int qy = y - 1 + rr;
                    if (qy < 0 || qy >= H) continue;
                    const uint32_t pa = (uint32_t)qy * W + (uint32_t)xlo;
                    const uint32_t wa = pa >> 6, sh = pa & 63u;
                    const uint64_t b0 = bm[wa];
                    uint64_t bits = b0 >> sh;
                    if (sh > 61u && (int)wa + 1 < bm64) bits |= bm[wa + 1] << (64u - sh);
                    uint32_t need = (uint32_t)bits & rowmask;
                    if (!need) continue;
                    const int rk0 = (int)(wpre[wa] + (uint32_t)__popcll(b0 & ((1ull << sh) - 1ull)));
                    const int s0 = pstart[rk0];
                    const int s1 = pstart[rk0 + __popc(need)];
                    for (int j = s0; j < s1 && need; j++) {
                        const uint2 e = csr[j];
                        const int u = (int)(e.y & 0xFFFFu);
                        const uint32_t dx = ((e.y >> 16) - (uint32_t)xlo) & 3u;
                        if (((need >> dx) & 1u) && u < i && ti - e.x <= dt32) {
                            need &= ~(1u << dx);
#pragma unroll
                            for (int c = 0; c < 3; c++)
                                if ((uint32_t)c == dx) cand[rr * 3 + c] = u;
                        }
                    }
                }
            }
            __syncthreads();  // the CSR is read no more
            // ---- the joins in the LDS forest (roots are the earliest slots):
            // hang under the smallest candidate, then hook roots in rounds
            if (t < tr.count) {
                int mn = i;
#pragma unroll
                for (int k = 0; k < 9; k++)
                    if (cand[k] >= 0 && cand[k] < mn) mn = cand[k];
                l_par[i] = mn;
            }
            __syncthreads();
            while (true) {
                for (int x = t; x < L; x += kWideThreads) {
                    int p = l_par[x];
                    while (true) {
                        const int g = l_par[p];
                        if (g == p) break;
                        l_par[x] = g;
                        p = g;
                    }
                }
                __syncthreads();
                bool changed = false;
                if (t < tr.count) {
                    const int pi = l_par[i];
#pragma unroll
                    for (int k = 0; k < 9; k++) {
                        if (cand[k] < 0) continue;
                        const int pc = l_par[cand[k]];
                        if (pc != pi) {
                            atomicMin(&l_par[pc > pi ? pc : pi], pc > pi ? pi : pc);
                            changed = true;
                        } else {
                            cand[k] = -1;  // joined (see link_union_publish)
                        }
                    }
                }
                if (!__syncthreads_or(changed)) break;
            }
            // ---- smallest input index per local tree; every slot joins it
            // through the global union-find (compare-and-swap only)
            for (int x = t; x < L; x += kWideThreads) minidx[x] = 0x7FFFFFFF;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kWidePer; k++) {
                const int a = t + k * kWideThreads;
                if (a < L) atomicMin(&minidx[l_par[a]], sid[k]);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kWidePer; k++) {
                const int a = t + k * kWideThreads;
                if (a < L) {
                    const int32_t m = minidx[l_par[a]];
                    if (m != sid[k]) gunion(w.gparent, sid[k], m, &w.status->err_internal);
                }
            }
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

hipError_t launch_link_wide(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_wide", s);
    const uint64_t pixels = (uint64_t)w.width * w.height;
    const int bm64 = pixels <= kLinkMaxPixels ? (int)((pixels + 63) / 64) : 0;
    const size_t dyn = (size_t)bm64 * 8 + (((size_t)bm64 * 2 + 7) & ~(size_t)7);
    // a tile per work-group and pass; few tiles overflow, so a small input
    // gets a small grid (the launch costs less when nothing overflows)
    const int pg = persistent_grid();
    const int want = (w.n_link_tiles + 3) / 4;
    const int grid = want < 1 ? 1 : want > pg ? pg : want;
    hipLaunchKernelGGL(k_link_wide, dim3(grid), dim3(kWideThreads), dyn, s, w, bm64);
    return hipGetLastError();
}

// ------------------------------------------- link fallback (big halos)
// Only the hits that a deep tile can join are sorted: the union of the deep
// tiles' windows, each window running from the first hit within dt before
// the tile's first hit (in its chunk) to the tile's end.  Windows grow with
// the tile index, so each deep tile adds one run of sorted positions to the
// union, starting at run_base, which lands at run_off in the sort's input.
// The hits are sorted by (pixel, sorted position); for each hit of a deep
// tile and each of its 9 pixels, the latest earlier hit at that pixel is the
// entry just before (pixel, own position), found by one binary search over
// all entries (the three pixels of a neighbour row side by side), and it is
// joined if it lies within dt.  Any hit of that pixel that is within dt lies
// in the tile's window, so the union holds it.
static_assert(kFbBlock >= kFbThreads + 1, "the plan keeps one value per thread in the radix LDS arrays");
struct PixSortJob {
    static constexpr bool kKeepSorted = true;
    Work w;
    __device__ int64_t count() const { return w.n; }
    // Position of the i-th element of the union: the last run starting at or
    // before i, searched between the runs holding the first elements of i's
    // radix block and of the next one.
    __device__ void load(int64_t i, uint64_t& k, uint32_t& v) const
    {
        const int64_t blk = i / kFbBlock;
        int a = w.blk_run[blk], b = w.blk_run[blk + 1] + 1;
        if (a < 0 || b <= a || b > w.status->n_deep) {
            atomicOr(&w.status->err_internal, 1);
            a = 0;
            b = 1;
        }
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (w.run_off[m] <= i) a = m; else b = m;
        }
        int64_t p = (int64_t)w.run_base[a] + (i - w.run_off[a]);
        if (w.run_off[a] > i || w.run_off[a + 1] <= i || p < 0 || p >= w.n) {
            atomicOr(&w.status->err_internal, 1);
            p = 0;
        }
        const uint32_t xy = w.s_xy[p];
        k = (uint64_t)(xy >> 16) * w.width + (xy & 0xFFFFu);
        v = (uint32_t)p;
    }
    __device__ int plan(RadixState& st, RadixLds& L)
    {
        const int t = threadIdx.x;
        const int nd = w.status->n_deep;
        if (nd <= 0 || w.status->err_range) return 0;  // st.active stays 0
        const int nt = w.n_link_tiles;
        // window start of every deep tile; -1 marks the others
        for (int k = t; k < nt; k += kFbThreads) w.deep_ws[k] = -1;
        __syncthreads();
        for (int q = t; q < nd; q += kFbThreads) {
            const int tile = w.deep_tiles[q];
            if (tile < 0 || tile >= nt) {
                atomicOr(&w.status->err_internal, 1);
                continue;
            }
            const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
            const uint64_t lo = sat_sub_u64(w.s_toa[tr.start], seg_dt(w, tr.seg));
            int64_t a = tr.seg_start, b = tr.start;
            while (a < b) {
                const int64_t m = (a + b) >> 1;
                if (w.s_toa[m] < lo) a = m + 1; else b = m;
            }
            w.deep_ws[tile] = (int32_t)a;
        }
        __syncthreads();
        // each thread takes a contiguous run of tiles; first the end of the
        // last deep tile before its run (a max-scan of the runs' last ends)
        const int per = (nt + kFbThreads - 1) / kFbThreads;
        const int k0 = t * per < nt ? t * per : nt;
        const int k1 = k0 + per < nt ? k0 + per : nt;
        int32_t* lend = reinterpret_cast<int32_t*>(L.k0);  // kFbThreads entries each
        int32_t* lsum = reinterpret_cast<int32_t*>(L.k1);
        int32_t* lcnt = reinterpret_cast<int32_t*>(L.key);  // kFbThreads + 1 entries
        int64_t last = -1;
        for (int k = k0; k < k1; k++)
            if (w.deep_ws[k] >= 0) {
                const TileRange tr = tile_range(w, kLinkKind, k, kLinkTile);
                last = tr.start + tr.count;
            }
        lend[t] = (int32_t)last;
        __syncthreads();
        if (t == 0) {
            int32_t run = -1;
            for (int i = 0; i < kFbThreads; i++) {
                const int32_t e = lend[i];
                lend[i] = run;
                run = e > run ? e : run;
            }
        }
        __syncthreads();
        const int64_t prev0 = lend[t];
        // positions each deep tile adds to the union; the thread's deep tiles
        int64_t prev = prev0, sum = 0;
        int32_t cnt = 0;
        for (int k = k0; k < k1; k++) {
            const int64_t ws = w.deep_ws[k];
            if (ws < 0) continue;
            const TileRange tr = tile_range(w, kLinkKind, k, kLinkTile);
            const int64_t base = ws > prev ? ws : prev;
            sum += tr.start + tr.count - base;
            prev = tr.start + tr.count;
            cnt++;
        }
        lsum[t] = (int32_t)sum;
        lcnt[t] = cnt;
        __syncthreads();
        if (t == 0) {
            int32_t run = 0, rr = 0;
            for (int i = 0; i < kFbThreads; i++) {
                const int32_t c = lsum[i], d = lcnt[i];
                lsum[i] = run;
                lcnt[i] = rr;
                run += c;
                rr += d;
            }
            L.misc = run;
            lcnt[kFbThreads] = rr;  // deep tiles counted (nd unless a listed tile was bad)
        }
        __syncthreads();
        const int nr = lcnt[kFbThreads];
        int64_t off = lsum[t];
        int r = lcnt[t];
        prev = prev0;
        for (int k = k0; k < k1; k++) {
            const int64_t ws = w.deep_ws[k];
            if (ws < 0) continue;
            const TileRange tr = tile_range(w, kLinkKind, k, kLinkTile);
            const int64_t base = ws > prev ? ws : prev;
            w.run_off[r] = (int32_t)off;
            w.run_base[r] = (int32_t)base;
            r++;
            off += tr.start + tr.count - base;
            prev = tr.start + tr.count;
        }
        if (t == 0) w.run_off[nr] = L.misc;
        __syncthreads();
        // the run holding the first element of every radix block
        const int64_t total = L.misc;
        const int nbk = (int)((total + kFbBlock - 1) / kFbBlock);
        for (int q = t; q < nr; q += kFbThreads) {
            const int64_t b0 = ((int64_t)w.run_off[q] + kFbBlock - 1) / kFbBlock;
            const int64_t b1 = ((int64_t)w.run_off[q + 1] + kFbBlock - 1) / kFbBlock;
            for (int64_t b = b0; b < b1; b++) w.blk_run[b] = q;
        }
        if (t == 0) w.blk_run[nbk] = nr > 0 ? nr - 1 : 0;
        if (t == 0) {
            st.active = nr > 0 ? 1 : 0;
            st.key_min = 0;
            const uint64_t top = (uint64_t)w.width * w.height - 1;
            const int bits = top == 0 ? 0 : 64 - __builtin_clzll(top);
            st.passes = bits <= 8 ? 1 : (bits + 7) / 8;
            st.n_eff = (int32_t)total;
        }
        __threadfence();  // the tables are read by every work-group once the plan is published
        return nd;
    }
    __device__ void store(int64_t, uint64_t, uint32_t) const {}
    // One extra task per deep tile.
    __device__ void extra(int e, const uint64_t* keys, const uint32_t* vals, RadixLds&)
    {
        RadixState& st = w.status->rs[1];
        const int64_t ne = st.n_eff;
        const int tile = w.deep_tiles[e];
        if (ne <= 0 || tile < 0 || tile >= w.n_link_tiles) {  // a bad entry is flagged by the plan
            signal_done(&st.query_done);
            return;
        }
        const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
        const int64_t p0 = tr.start;
        const int64_t p1 = tr.start + tr.count;
        const uint64_t dt = seg_dt(w, tr.seg);
        const int32_t n1 = (int32_t)ne;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += kFbThreads) {
            const uint32_t xy = w.s_xy[p];
            const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
            const uint64_t toa = w.s_toa[p];
            // one neighbour row at a time, its three pixels side by side
            for (int dy = -1; dy <= 1; dy++) {
                const int qy = y + dy;
                if (qy < 0 || qy >= (int)w.height) continue;
                uint32_t key[3];
                int32_t a[3], b[3];
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    const int qx = x + d - 1;
                    const bool in = qx >= 0 && qx < (int)w.width;
                    key[d] = in ? (uint32_t)qy * w.width + (uint32_t)qx : 0u;  // below 2^32: 16-bit coordinates
                    a[d] = 0;
                    b[d] = in ? n1 : 0;
                }
                // first entry not before (pixel, p), the three searches in
                // lockstep with every load issued (a finished search reads a
                // valid entry and keeps its bounds)
                for (int32_t span = n1; span > 0; span >>= 1) {
                    uint64_t km[3];
                    uint32_t vm[3];
                    int32_t mm[3];
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        const int32_t m = (a[d] + b[d]) >> 1;
                        mm[d] = m < n1 ? m : n1 - 1;
                        km[d] = keys[mm[d]];
                        vm[d] = vals[mm[d]];
                    }
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        const bool go = a[d] < b[d];
                        const bool before = km[d] < key[d] || (km[d] == key[d] && (int64_t)vm[d] < p);
                        a[d] = go && before ? mm[d] + 1 : a[d];
                        b[d] = go && !before ? mm[d] : b[d];
                    }
                }
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    if (a[d] == 0 || keys[a[d] - 1] != key[d]) continue;  // outside, or nothing before
                    const int64_t c = vals[a[d] - 1];
                    if (c < 0 || c >= p) {
                        atomicOr(&w.status->err_internal, 1);
                    } else if (c >= tr.seg_start && toa - w.s_toa[c] <= dt) {
                        gunion(w.gparent, w.s_idx[c], w.s_idx[p], &w.status->err_internal);
                    }
                }
            }
        }
        signal_done(&st.query_done);
    }
};

__global__ __launch_bounds__(kFbThreads) void k_link_fallback(Work w)
{
    resolve_count(w);
    if (!w.status->n_deep || w.status->err_range) return;  // the common case
    PixSortJob job{w};
    uint64_t* kb[2] = {w.fb_key[0], w.fb_key[1]};
    uint32_t* vb[2] = {w.fb_val[0], w.fb_val[1]};
    radix_engine(job, &w.status->rs[1], kb, vb, w.fb_hist, w.n_fb_blocks, &w.status->err_internal);
}



hipError_t launch_link_fallback(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_fallback", s);
    hipLaunchKernelGGL(k_link_fallback, dim3(persistent_grid()), dim3(kFbThreads), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------- cross-tile unions
// Cross-tile unions: one wave per link tile's edge region, all tiles in one
// pass (the regions hold a handful of edges, so the time is the latency of
// reading the count, the edges and the parent chains once).
__global__ __launch_bounds__(256) void k_union_edges(Work w)
{
    resolve_count(w);
    if (w.status->err_range) return;
    const int64_t k = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (k >= w.n_link_tiles) return;
    const int ne = w.tile_nedge[k];
    for (int e = threadIdx.x & (kWave - 1); e < ne; e += kWave) {
        const int2 ed = w.edges[k * kLinkHaloCap + e];
        gunion(w.gparent, ed.x, ed.y, &w.status->err_internal);
    }
}

hipError_t launch_union_edges(const Work& w, hipStream_t s)
{
    TimedLaunch tl("union_edges", s);
    const int per = 256 / kWave;
    const int grid = w.n_link_tiles > 0 ? (w.n_link_tiles + per - 1) / per : 1;
    hipLaunchKernelGGL(k_union_edges, dim3(grid), dim3(256), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------------------ flatten
// labels[i] = root(i) (minus the chunk's first index for a batch, whose
// labels are chunk-local).  One work-group per block of kScanBlock indices; a
// root (root(i) == i) is a cluster: its bit is set in the block's mask and
// the block's root count is stored for the compaction scan.
__global__ __launch_bounds__(kScanThreads) void k_flatten(Work w, int32_t* __restrict__ labels)
{
    static_assert(kScanBlock == 8 * kScanThreads && kScanThreads % kWave == 0, "mask layout");
    static_assert(kScanBlock / 64 <= kWave, "one wave scans the block's mask words");
    __shared__ uint32_t wsum[kScanThreads / kWave];
    __shared__ uint32_t s_wc[kScanBlock / 64];  // roots per mask word
    resolve_count(w);
    if (w.status->err_range || (int)blockIdx.x >= w.n_scan_blocks) return;
    const int b = blockIdx.x;
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    const TileRange tr = tile_range(w, kScanKind, b, kScanBlock);
    const int64_t base = tr.start;
    const int64_t end = tr.start + tr.count;
    const int64_t lab0 = w.n_seg > 1 ? tr.seg_start : 0;  // a batch's labels are chunk-local
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kScanBlock / kScanThreads; q++) {
        const int64_t i = base + q * kScanThreads + t;
        bool root = false;
        if (i < end) {
            const int32_t r = gfind_final(w.gparent, (int32_t)i, &w.status->err_internal);
            labels[i] = r - (int32_t)lab0;
            root = (r == (int32_t)i);
        }
        const unsigned long long m = __ballot(root);
        if (lane == 0) {
            w.root_mask[(int64_t)b * (kScanBlock / 64) + q * (kScanThreads / kWave) + wid] = m;
            s_wc[q * (kScanThreads / kWave) + wid] = (uint32_t)__popcll(m);
        }
        c += root;
    }
    uint32_t total;
    block_exclusive_scan<kScanThreads>(c, wsum, &total);  // (its barriers also publish s_wc)
    if (t == 0) w.blk_count[b] = total;
    if (wid == 0) {  // roots in the block's earlier mask words, for rank lookups
        const uint32_t v = lane < kScanBlock / 64 ? s_wc[lane] : 0u;
        const uint32_t ex = wave_incl_scan_u32(v) - v;
        if (lane < kScanBlock / 64) w.root_wpre[(int64_t)b * (kScanBlock / 64) + lane] = (uint16_t)ex;
    }
}

hipError_t launch_flatten(const Work& w, int32_t* labels, hipStream_t s)
{
    TimedLaunch tl("flatten", s);
    hipLaunchKernelGGL(k_flatten, dim3(w.n_scan_blocks), dim3(kScanThreads), 0, s, w, labels);
    return hipGetLastError();
}

}  // namespace hc
