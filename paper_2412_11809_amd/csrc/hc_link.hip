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
//   * an occupancy bitmap of the sensor and the popcount prefix of its words
//     give every occupied pixel of the tile a dense rank, and a CSR lists the
//     tile's hits per pixel rank in time order -- the tile-sized replacement
//     of the paper's dense matrix;
//   * each tile hit joins, at each of its 9 pixels, the latest earlier hit if
//     it lies within dt (the hit the paper's matrix holds).  Hits of one pixel
//     whose consecutive ToAs differ by <= dt are chained by their own-pixel
//     probes, so this reaches every earlier hit within dt;
//   * the joins are applied in bulk rounds in an LDS forest whose roots are
//     the earliest slots (the paper's time-ordered roots); the smallest input
//     index of every tree is the label candidate written to the global parent
//     array, and halo hits joined by the tile are queued as cross-tile edges.
// A tile whose halo does not fit (or whose ToA span exceeds 32 bits) is
// handled by k_link_fallback: a pixel-sorted copy of all hits plus binary
// searches.  k_union_edges applies the queued cross-tile edges with atomic
// compare-and-swap, and k_flatten writes labels[i] = root(i).
#include "hc_device.h"
#include "hc_radix.h"

namespace hc {

// Which neighbour search runs: 0 = window scan only (k_link_window),
// 1 = per tile, window scan or pixel index (k_link), 2 = pixel index only
// (k_link).  The window scan needs coordinates below 2^14, the pixel index
// room for the sensor's occupancy bitmap in LDS.
enum { kLinkWindowOnly = 0, kLinkHybrid = 1, kLinkIndexOnly = 2 };
__host__ __device__ inline int link_kernel(const Work& w)
{
    const bool win_ok = w.width <= kLinkWindowMaxDim && w.height <= kLinkWindowMaxDim;
    const bool idx_ok = (uint64_t)w.width * w.height <= kLinkMaxPixels;
    if (w.link_mode == 1 || !win_ok) return kLinkIndexOnly;
    if (w.link_mode == 2 || !idx_ok) return kLinkWindowOnly;
    // beyond 256 x 256 pixels the bitmap leaves room for one work-group per
    // CU, which costs every tile more than scanning its windows
    if (w.link_mode == 0 && (uint64_t)w.width * w.height > kLinkHybridMaxPixels) return kLinkWindowOnly;
    return kLinkHybrid;
}

// First halo position of every link tile: the earliest sorted position p
// with toa(p) >= toa(p0) - dt (a suffix of the positions before p0, so a
// binary search), or -1 when the halo exceeds kLinkHaloCap, the tile's ToA
// span does not fit 32 bits or the sensor is too large for the LDS pixel
// bitmap (such tiles go to the fallback).
__global__ void k_link_halo(Work w)
{
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
    overflow |= link_kernel(w) != kLinkWindowOnly && (uint64_t)w.width * w.height > kLinkMaxPixels;  // no bitmap room
    w.link_h0[k] = overflow ? -1 : (int32_t)a;
}

hipError_t launch_link_halo(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_halo", s);
    hipLaunchKernelGGL(k_link_halo, dim3((w.n_link_tiles + 255) / 256), dim3(256), 0, s, w);
    return hipGetLastError();
}

// Joins of one tile (cand: per tile hit, the slot joined at each of its 9
// pixels, or -1) applied in bulk rounds in the LDS forest l_par: hook every
// edge's larger root under the smaller (atomic minimum), then jump pointers
// until every tree is a star; repeat until no edge joins two roots.  Then the
// smallest input index of every local tree is published: as the parent of
// the tree's tile hits, and as cross-tile edges for its halo hits.
// minidx: LDS scratch of L words (the caller's ToA array, no longer read).
template <int PER, int LPER>
__device__ inline void link_union_publish(const Work& w, int tile, int32_t* l_par, int (&cand)[PER][9],
                                          const int32_t (&ids)[LPER], int hl, int L, int32_t* minidx)
{
    const int t = threadIdx.x;
    while (true) {
        bool changed = false;
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int i = hl + t + q * kLinkThreads;
            if (i >= L) continue;
            const int pi = l_par[i];
#pragma unroll
            for (int k = 0; k < 9; k++) {
                if (cand[q][k] < 0) continue;
                const int pc = l_par[cand[q][k]];
                if (pc != pi) {
                    atomicMin(&l_par[pc > pi ? pc : pi], pc > pi ? pi : pc);
                    changed = true;
                }
            }
        }
        __syncthreads();
        for (int x = t; x < L; x += kLinkThreads) {
            int p = l_par[x];
            while (true) {
                const int g = l_par[p];
                if (g == p) break;
                p = g;
            }
            l_par[x] = p;
        }
        if (!__syncthreads_or(changed)) break;
    }

    // ---- smallest input index per local tree, then publish
    for (int i = t; i < L; i += kLinkThreads) minidx[i] = 0x7FFFFFFF;
    __syncthreads();
    int32_t root[LPER];
#pragma unroll
    for (int q = 0; q < LPER; q++) {
        const int i = t + q * kLinkThreads;
        root[q] = i < L ? l_par[i] : -1;
        if (root[q] >= 0) atomicMin(&minidx[root[q]], ids[q]);
    }
    __syncthreads();
    // halo hits joined by this tile become cross-tile edges, in the tile's
    // own region of kLinkHaloCap entries (positions from a block scan)
    int32_t m[LPER];
    uint32_t ne = 0;
#pragma unroll
    for (int q = 0; q < LPER; q++) {
        const int i = t + q * kLinkThreads;
        m[q] = i < L ? minidx[root[q]] : -1;
        ne += (i < hl && ids[q] != m[q]) ? 1u : 0u;
    }
    __shared__ uint32_t e_wsum[kLinkThreads / kWave];
    uint32_t n_tile_edges;
    uint32_t pos = block_exclusive_scan<kLinkThreads>(ne, e_wsum, &n_tile_edges);
    if (t == 0) w.tile_nedge[tile] = (int32_t)n_tile_edges;
    const int64_t e_base = (int64_t)tile * kLinkHaloCap;
#pragma unroll
    for (int q = 0; q < LPER; q++) {
        const int i = t + q * kLinkThreads;
        if (i >= L) continue;
        if (i >= hl) {
            w.gparent[ids[q]] = m[q];
        } else if (ids[q] != m[q]) {
            w.edges[e_base + pos++] = make_int2(ids[q], m[q]);  // pos < hl <= kLinkHaloCap
        }
    }
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

// One work-group per tile of kLinkTile sorted hits (+ halo), all in LDS.
//
// Local slots 0..L-1 are the sorted positions h0..p1-1, so a smaller slot is
// an earlier hit.  The paper's per-pixel "last hit" matrix is replaced by a
// tile-sized index of the occupied pixels:
//   * an occupancy bitmap of the sensor plus the popcount prefix of its words
//     gives every occupied pixel a dense rank (pixel order) without hashing;
//   * a CSR lists, per occupied pixel, the slots of its hits in ascending
//     order, so the three pixels of a neighbour row are three consecutive
//     segments and the latest earlier hit at a pixel is found by stepping back
//     from its segment's end (usually one step).
// Each tile hit joins, for each of its (up to) 9 neighbour pixels, the latest
// earlier hit there if it lies within dt -- the hit the paper's matrix would
// hold.  Joins are applied in bulk rounds (hook the larger root under the
// smaller with an atomic minimum, then jump pointers until every tree is a
// star) in an LDS forest whose roots are the earliest slots, as in the paper's
// time-ordered forest.  The smallest input index of every local tree is then
// published as the label candidate of its tile hits; halo hits joined by the
// tile become cross-tile edges.
// Dynamic LDS: bitmap (bm_words words) followed by the 16-bit word prefix
// counts.  LDS is kept near 53 KiB (256 x 256 sensor) so three work-groups
// share a CU.
__global__ __launch_bounds__(kLinkThreads) void k_link(Work w, int bm_words)
{
    constexpr int LCAP = kLinkTile + kLinkHaloCap;
    constexpr int PER = kLinkTile / kLinkThreads;
    constexpr int LPER = LCAP / kLinkThreads;
    constexpr uint16_t kUnsorted = 0x8000u;
    __shared__ uint32_t l_toa[LCAP];
    __shared__ uint32_t l_xy[LCAP];
    __shared__ int32_t l_par[LCAP];
    __shared__ uint16_t l_rank[LCAP];     // hit's rank among its pixel's hits, then root
    __shared__ uint16_t l_pixr[LCAP];     // hit's pixel rank
    __shared__ uint16_t csr[LCAP];        // slots grouped by pixel rank
    __shared__ uint16_t pstart[LCAP + 2]; // count (packed in pairs), then first CSR position per pixel rank [| kUnsorted]
    __shared__ uint32_t wsum[kLinkThreads / kWave];
    __shared__ uint32_t s_cost;
    extern __shared__ uint32_t dyn[];
    uint32_t* bm = dyn;
    uint16_t* wpre = reinterpret_cast<uint16_t*>(dyn + bm_words);
    uint32_t* pcount = reinterpret_cast<uint32_t*>(pstart);  // two 16-bit counters per word

    if (w.status->err_range) return;
    const int tile = xcd_tile(w.n_link_tiles, w.xcd_map);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
    const int64_t p0 = tr.start;
    const int64_t p1 = tr.start + tr.count;
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
            w.tile_nedge[tile] = 0;
        }
        return;
    }
    const int L = (int)(p1 - h0);
    const int hl = (int)(p0 - h0);
    const uint64_t tbase = w.s_toa[h0];
    const uint32_t W = w.width;
    int32_t ids[LPER];
#pragma unroll
    for (int q = 0; q < LPER; q++) {
        const int i = t + q * kLinkThreads;
        ids[q] = -1;
        if (i < L) {
            const int64_t p = h0 + i;
            l_toa[i] = (uint32_t)(w.s_toa[p] - tbase);
            l_xy[i] = w.s_xy[p];
            l_par[i] = i;
            int32_t id = w.s_idx[p];
            if (id < 0 || id >= w.n) {
                atomicOr(&w.status->err_internal, 1);
                id = 0;
            }
            ids[q] = id;
        }
    }
    if (t == 0) s_cost = 0u;
    __syncthreads();

    // ---- the dt window of every tile hit (slots [lo, i)) and what scanning
    // the windows would cost: per wave, the longest window of each step
    const uint64_t dt = seg_dt(w, tr.seg);
    const int lane = t & (kWave - 1);
    int lo[PER];
    uint32_t cost = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = hl + t + q * kLinkThreads;
        lo[q] = i;
        if (i < L) {
            const uint32_t ti = l_toa[i];
            int a = 0;
            if (dt < (uint64_t)ti) {
                const uint32_t th = ti - (uint32_t)dt;
                int b = i;
                while (a < b) {
                    const int m = (a + b) >> 1;
                    if (l_toa[m] < th) a = m + 1; else b = m;
                }
            }
            lo[q] = a;
        }
        uint32_t win = (uint32_t)(i < L ? i - lo[q] : 0);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t v = __shfl_xor(win, o, kWave);
            win = v > win ? v : win;
        }
        cost += win;
    }
    if (lane == 0) atomicAdd(&s_cost, cost * kWave);
    __syncthreads();
    // short windows (sparse hits): scan them; long ones (showers): pixel index
    const bool window = link_kernel(w) == kLinkHybrid && s_cost <= (uint32_t)(kLinkWindowMeanCost * (L - hl));
    int cand[PER][9];
    if (window) {
        link_window_search<PER>(l_toa, l_xy, hl, L, lo, cand);
    } else {
    for (int i = t; i < bm_words; i += kLinkThreads) bm[i] = 0u;
    for (int i = t; i < (LCAP + 2) / 2; i += kLinkThreads) pcount[i] = 0u;
    __syncthreads();

    // ---- occupancy bitmap
    for (int i = t; i < L; i += kLinkThreads) {
        const uint32_t xy = l_xy[i];
        const uint32_t pix = (xy >> 16) * W + (xy & 0xFFFFu);
        atomicOr(&bm[pix >> 5], 1u << (pix & 31u));
    }
    __syncthreads();
    // ---- popcount prefix of the bitmap words (rank of the first pixel of a word)
    {
        const int per = (bm_words + kLinkThreads - 1) / kLinkThreads;
        const int w0 = t * per;
        uint32_t c = 0;
        for (int k = 0; k < per; k++)
            if (w0 + k < bm_words) c += __popc(bm[w0 + k]);
        uint32_t run = block_exclusive_scan<kLinkThreads>(c, wsum, nullptr);
        for (int k = 0; k < per; k++)
            if (w0 + k < bm_words) {
                wpre[w0 + k] = (uint16_t)run;
                run += __popc(bm[w0 + k]);
            }
    }
    __syncthreads();
    // ---- per-pixel counts (the atomic returns each hit's rank in its pixel)
    for (int i = t; i < L; i += kLinkThreads) {
        const uint32_t xy = l_xy[i];
        const uint32_t pix = (xy >> 16) * W + (xy & 0xFFFFu);
        const uint32_t wd = pix >> 5;
        const uint32_t r = wpre[wd] + __popc(bm[wd] & ((1u << (pix & 31u)) - 1u));
        l_pixr[i] = (uint16_t)r;
        const uint32_t half = 16u * (r & 1u);  // counts stay below 2^16: no carry into the neighbour
        l_rank[i] = (uint16_t)(atomicAdd(&pcount[r >> 1], 1u << half) >> half);
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
        if (t == kLinkThreads - 1) pstart[LCAP] = (uint16_t)run;
    }
    __syncthreads();
    for (int i = t; i < L; i += kLinkThreads) csr[pstart[l_pixr[i]] + l_rank[i]] = (uint16_t)i;
    __syncthreads();
    // ---- sort every pixel's segment by slot (segments are short; a pile-up
    // of more than 64 hits on one pixel is left unsorted and scanned instead)
    for (int r = t; r < LCAP; r += kLinkThreads) {
        // a neighbouring thread may already have flagged pstart[r + 1]
        const int s0 = (int)(pstart[r] & ~kUnsorted), s1 = (int)(pstart[r + 1] & ~kUnsorted);
        const int cnt = s1 - s0;
        if (cnt < 2) continue;
        if (cnt > 64) {
            pstart[r] = (uint16_t)(s0 | kUnsorted);
            continue;
        }
        for (int a = s0 + 1; a < s1; a++) {
            const uint16_t v = csr[a];
            int b = a - 1;
            while (b >= s0 && csr[b] > v) {
                csr[b + 1] = csr[b];
                b--;
            }
            csr[b + 1] = v;
        }
    }
    __syncthreads();

    // ---- neighbour search: latest earlier hit per neighbour pixel
    const int H = (int)w.height;
#pragma unroll
    for (int q = 0; q < PER; q++) {
#pragma unroll
        for (int k = 0; k < 9; k++) cand[q][k] = -1;
        const int i = hl + t + q * kLinkThreads;
        if (i >= L) continue;
        const uint32_t xy = l_xy[i];
        const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
        const uint32_t ti = l_toa[i];
        const int xlo = x > 0 ? x - 1 : 0;
        const int xhi = x + 1 < (int)W ? x + 1 : (int)W - 1;
        const uint32_t rowmask = (1u << (xhi - xlo + 1)) - 1u;
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const int qy = y - 1 + r;
            if (qy < 0 || qy >= H) continue;
            const uint32_t pa = (uint32_t)qy * W + (uint32_t)xlo;
            const uint32_t wa = pa >> 5, sh = pa & 31u;
            uint64_t bits = bm[wa];
            if (sh > 29u && wa + 1 < (uint32_t)bm_words) bits |= (uint64_t)bm[wa + 1] << 32;
            const uint32_t occ = (uint32_t)(bits >> sh) & rowmask;
            if (!occ) continue;
            // rank of the first occupied pixel of this row segment
            int rk = (int)(wpre[wa] + __popc(bm[wa] & ((1u << sh) - 1u)));
#pragma unroll
            for (int k = 0; k < 3; k++) {
                if (!(occ & (1u << k))) continue;
                const uint32_t st = pstart[rk];  // (16-bit entry)
                const int s0 = (int)(st & ~kUnsorted), s1 = (int)(pstart[rk + 1] & ~kUnsorted);
                rk++;
                int a = -1;
                if (!(st & kUnsorted)) {
                    int j = s1 - 1;
                    while (j >= s0 && (int)csr[j] >= i) j--;
                    if (j >= s0) a = csr[j];
                } else {
                    for (int j = s0; j < s1; j++) {
                        const int v = csr[j];
                        if (v < i && v > a) a = v;
                    }
                }
                if (a >= 0 && (uint64_t)(ti - l_toa[a]) <= dt) {
#pragma unroll
                    for (int kk = 0; kk < 9; kk++)
                        if (kk == 3 * r + k) cand[q][kk] = a;
                }
            }
        }
    }

    }  // pixel index
    link_union_publish(w, tile, l_par, cand, ids, hl, L, reinterpret_cast<int32_t*>(l_toa));
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
__global__ __launch_bounds__(kLinkThreads) void k_link_window(Work w)
{
    constexpr int LCAP = kLinkTile + kLinkHaloCap;
    constexpr int PER = kLinkTile / kLinkThreads;
    constexpr int LPER = LCAP / kLinkThreads;
    __shared__ uint32_t l_toa[LCAP];
    __shared__ uint32_t l_xy[LCAP];
    __shared__ int32_t l_par[LCAP];

    if (w.status->err_range) return;
    const int tile = xcd_tile(w.n_link_tiles, w.xcd_map);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
    const int64_t p0 = tr.start;
    const int64_t p1 = tr.start + tr.count;
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
            w.tile_nedge[tile] = 0;
        }
        return;
    }
    const int L = (int)(p1 - h0);
    const int hl = (int)(p0 - h0);
    const uint64_t tbase = w.s_toa[h0];
    int32_t ids[LPER];
#pragma unroll
    for (int q = 0; q < LPER; q++) {
        const int i = t + q * kLinkThreads;
        ids[q] = -1;
        if (i < L) {
            const int64_t p = h0 + i;
            l_toa[i] = (uint32_t)(w.s_toa[p] - tbase);
            l_xy[i] = w.s_xy[p];
            l_par[i] = i;
            int32_t id = w.s_idx[p];
            if (id < 0 || id >= w.n) {
                atomicOr(&w.status->err_internal, 1);
                id = 0;
            }
            ids[q] = id;
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
    link_union_publish(w, tile, l_par, cand, ids, hl, L, reinterpret_cast<int32_t*>(l_toa));
}

// The window-scan kernel, or the per-tile hybrid / pixel-index kernel.
hipError_t launch_link(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link", s);
    const dim3 grid(xcd_grid(w.n_link_tiles));
    if (link_kernel(w) == kLinkWindowOnly) {
        hipLaunchKernelGGL(k_link_window, grid, dim3(kLinkThreads), 0, s, w);
    } else {
        const int bm_words = link_bitmap_words(w.width, w.height);
        const size_t dyn = (size_t)bm_words * 4 + (((size_t)bm_words * 2 + 3) & ~(size_t)3);
        hipLaunchKernelGGL(k_link, grid, dim3(kLinkThreads), dyn, s, w, bm_words);
    }
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
        const TileRange tr = tile_range(w, kLinkKind, tile, kLinkTile);
        const int64_t p0 = tr.start;
        const int64_t p1 = tr.start + tr.count;
        const uint64_t dt = seg_dt(w, tr.seg);
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
                        } else if (c >= tr.seg_start && toa - w.s_toa[c] <= dt) {
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



hipError_t launch_link_fallback(const Work& w, hipStream_t s)
{
    TimedLaunch tl("link_fallback", s);
    hipLaunchKernelGGL(k_link_fallback, dim3(persistent_grid()), dim3(kFbThreads), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------- cross-tile unions
// Cross-tile unions: one work-group per link tile's edge region (grid-stride).
__global__ __launch_bounds__(64) void k_union_edges(Work w)
{
    if (w.status->err_range) return;
    for (int64_t k = blockIdx.x; k < w.n_link_tiles; k += gridDim.x) {
        const int ne = w.tile_nedge[k];
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            const int2 ed = w.edges[k * kLinkHaloCap + e];
            gunion(w.gparent, ed.x, ed.y, &w.status->err_internal);
        }
    }
}

hipError_t launch_union_edges(const Work& w, hipStream_t s)
{
    TimedLaunch tl("union_edges", s);
    const int grid = w.n_link_tiles < 8192 ? (w.n_link_tiles > 0 ? w.n_link_tiles : 1) : 8192;
    hipLaunchKernelGGL(k_union_edges, dim3(grid), dim3(64), 0, s, w);
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
    const TileRange tr = tile_range(w, kScanKind, b, kScanBlock);
    const int64_t base = tr.start;
    const int64_t end = tr.start + tr.count;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kScanBlock / kScanThreads; q++) {
        const int64_t i = base + q * kScanThreads + t;
        bool root = false;
        if (i < end) {
            const int32_t r = gfind_final(w.gparent, (int32_t)i, &w.status->err_internal);
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
