// Step A1 of the clustering path: order the hits by (ToA, input index).
//
// The paper sorts each buffer by ToA (radix sort, Step 3 of its high-level GPU
// algorithm) before the neighbour sweep, and relies on the stream being only
// partly unsorted ("t-ordered", Section 3.1).  Here that partial order is
// exploited directly:
//   k_tile_sort   sorts tiles of T consecutive input hits in LDS (stable radix
//                 sort on ToA relative to the tile minimum), writes the tile in
//                 sorted order plus its min/max keys and the last key of each
//                 of its kTileQ equal parts;
//   k_tile_rank   gives every element its global rank: all of its tile's
//                 predecessors plus, for each of the m neighbour tiles on both
//                 sides, the number of smaller keys there (a merge path of the
//                 two sorted tiles in LDS, over only the neighbour's parts that
//                 can interleave with this tile, found from their last keys;
//                 binary searches for short tiles), and writes the element's
//                 sorted record at that rank.
//                 This is exact whenever tiles more than m apart do not
//                 interleave, which the kernel verifies from the tile min/max
//                 keys: the max of tile i lies below the min of tile i+m+1,
//                 and the tile minima ascend from tile m+1 on (then every
//                 tile more than m places after tile i lies wholly above
//                 it, so every element of a tile more than m tiles away is
//                 smaller, resp. larger, than every element of this one); a
//                 displacement of at most m*T/2 positions guarantees it.
//                 The first m+1 tiles need no order among themselves.
//   k_sort_fallback  if any check failed (or a tile's ToA range exceeds 32
//                 bits), re-sorts everything with a ticketed LSD radix sort;
//                 otherwise it exits at once.
// Output: the sorted structure-of-arrays s_toa / s_xy / s_tot / s_idx.
#include "hc_device.h"
#include "hc_radix.h"

namespace hc {

// --------------------------------------------------------------- init
__global__ void k_init(Work w)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    int32_t* s = reinterpret_cast<int32_t*>(w.status);
    for (int i = t; i < (int)(sizeof(Status) / 4); i += stride) s[i] = 0;
    if (t == 0 && w.force_fallback) w.status->sort_fallback = 1;
}

hipError_t launch_init(const Work& w, hipStream_t s)
{
    TimedLaunch tl("init", s);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, w);
    return hipGetLastError();
}

// ---------------------------------------------------------- tile sort
// NT threads sort a tile of T = NT * IPT hits (8192-hit tiles use 1024
// threads: their LDS allows one work-group per CU, so it gets more waves).
template <int NT, int IPT>
__global__ __launch_bounds__(NT, NT == 512 ? 6 : 4) void k_tile_sort(const hc_hit* __restrict__ hits, Work w)
{
    resolve_count(w);
    constexpr int T = NT * IPT;
    __shared__ uint32_t kr[T];  // ToA - tile minimum, by input position
    __shared__ uint16_t e0[T], e1[T];
    __shared__ uint16_t cnt[16 * NT];
    __shared__ uint32_t wsum[NT / kWave];
    __shared__ uint64_t red[NT / kWave];

    const int tile = xcd_tile(w.n_sort_tiles, w.xcd_map);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const TileRange tr = tile_range(w, kSortKind, tile, T);
    const int64_t base = tr.start;
    const int cnt_e = tr.count;

    // ToAs first; the pixel (checked against the sensor) comes with the
    // payload once the tile is sorted
    uint64_t toa[IPT];
    uint64_t tmin = ~0ull, tmax = 0;
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const int e = t + j * NT;
        toa[j] = 0;
        if (e < cnt_e) {
            toa[j] = hits[base + e].toa;
            tmin = toa[j] < tmin ? toa[j] : tmin;
            tmax = toa[j] > tmax ? toa[j] : tmax;
        }
    }
    tmin = block_min_u64<NT>(tmin, red);
    tmax = block_max_u64<NT>(tmax, red);
    const uint64_t range = tmax - tmin;
    if (range > 0xFFFFFFFFull) {
        bool bad = false;
        for (int e = t; e < cnt_e; e += NT) bad |= (hits[base + e].x >= w.width) | (hits[base + e].y >= w.height);
        if (bad) atomicOr(&w.status->err_range, 1);
        if (t == 0) {
            TileInfo ti;
            ti.base = tmin;
            ti.max_toa = tmax;
            ti.min_idx = (int32_t)base;
            ti.max_idx = (int32_t)(base + cnt_e - 1);
            ti.wide = 1;
            ti.count = cnt_e;
            w.tiles[tile] = ti;
            atomicOr(&w.status->sort_fallback, 1);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const int e = t + j * NT;
        kr[e] = e < cnt_e ? (uint32_t)(toa[j] - tmin) : 0xFFFFFFFFu;
        e0[e] = (uint16_t)e;
    }
    __syncthreads();
    const int bits = range == 0 ? 0 : 32 - __builtin_clz((uint32_t)range);
    const int which = block_radix_sort_index<NT, IPT>(kr, e0, e1, cnt, wsum, bits);
    const uint16_t* sv = which ? e1 : e0;
    bool bad = false;
#pragma unroll 2
    for (int j = 0; j < IPT; j++) {
        const int e = t + j * NT;
        if (e < cnt_e) {
            uint16_t l = sv[e];
            if (l >= cnt_e) {
                atomicOr(&w.status->err_internal, 1);
                l = 0;
            }
            // the record's second half: x | y << 16, tot | reserved << 16
            const uint2 xyt = reinterpret_cast<const uint2*>(hits + base + l)[1];
            bad |= ((xyt.x & 0xFFFFu) >= w.width) | ((xyt.x >> 16) >= w.height);
            w.ts_rel[base + e] = kr[l];
            w.ts_pay[base + e] = make_uint2((uint32_t)l | (xyt.y << 16), xyt.x);
        }
    }
    if (bad) atomicOr(&w.status->err_range, 1);
    if (t < kTileQ) {  // the last key of each of the kTileQ parts
        const int S = (cnt_e + kTileQ - 1) / kTileQ;
        const int e = (t + 1) * S - 1 < cnt_e - 1 ? (t + 1) * S - 1 : cnt_e - 1;
        w.tile_q[(int64_t)tile * kTileQ + t] = kr[sv[e]];
    }
    if (t == 0) {
        TileInfo ti;
        ti.base = tmin;
        ti.max_toa = tmax;
        ti.min_idx = (int32_t)(base + sv[0]);
        ti.max_idx = (int32_t)(base + sv[cnt_e - 1]);
        ti.wide = 0;
        ti.count = cnt_e;
        w.tiles[tile] = ti;
    }
}

hipError_t launch_tile_sort(const hc_hit* hits, const Work& w, hipStream_t s)
{
    TimedLaunch tl("tile_sort", s);
    const dim3 grid(xcd_grid(w.n_sort_tiles));
    switch (w.sort_tile) {
    case 2048: hipLaunchKernelGGL((k_tile_sort<512, 4>), grid, dim3(512), 0, s, hits, w); break;
    case 4096: hipLaunchKernelGGL((k_tile_sort<512, 8>), grid, dim3(512), 0, s, hits, w); break;
    case 8192: hipLaunchKernelGGL((k_tile_sort<1024, 8>), grid, dim3(1024), 0, s, hits, w); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// --------------------------------------------------------- tile merge
// Number of elements of a sorted tile (keys rel[0..cnt) relative to base)
// smaller than key (toa, idx): elements of an earlier tile count when
// toa <= key toa (their indices are smaller), of a later tile when toa < key.
// Searches [lo, cnt) only: the caller's keys ascend, so counts do too.
__device__ inline int count_below(const uint32_t* rel, int cnt, uint64_t base, uint64_t toa,
                                  bool earlier, int lo)
{
    if (toa < base) return 0;
    const uint64_t d64 = toa - base;
    if (d64 > 0xFFFFFFFFull) return cnt;
    const uint32_t d = (uint32_t)d64;
    int a = lo, b = cnt;
    while (a < b) {
        const int m = (a + b) >> 1;
        const bool below = earlier ? (rel[m] <= d) : (rel[m] < d);
        if (below) a = m + 1; else b = m;
    }
    return a;
}

// LDS position of key e in the merge path's key arrays: the low three bits
// are XORed with bits 5..7, so the sequential merges of consecutive lanes,
// whose positions lie about eight keys apart, fall into different banks.
__device__ inline int merge_swz(int e) { return e ^ ((e >> 5) & 7); }

// Global rank of every element of tile j: all elements of tiles before
// j - m, its position in its own tile, and its count in each neighbour tile;
// the element's sorted record is written at that rank.  Also checks the
// conditions under which this is exact (if they fail anywhere, the fallback
// sort rewrites every record).
template <int IPT>
__global__ __launch_bounds__(kSortThreads) void k_tile_rank(Work w)
{
    resolve_count(w);
    constexpr int T = kSortThreads * IPT;
    static_assert(IPT % 4 == 0, "ranks are staged four at a time");
    __shared__ __align__(16) uint32_t nk[T];
    if (w.status->sort_fallback) return;  // a wide tile: everything is re-sorted later
    const int j = xcd_tile(w.n_sort_tiles, w.xcd_map);
    if (j < 0) return;
    const int t = threadIdx.x;
    const int m = w.sort_m;
    const TileInfo tj = w.tiles[j];
    // only tiles of the same chunk are merged; ranks are chunk-relative
    const TileRange jr = tile_range(w, kSortKind, j, T);
    const int t0 = jr.tile0, nt = jr.tile1;

    if (t == 0) {
        bool bad = false;
        // tile minima ascend from the chunk's tile m + 1 on (maxima need not:
        // a short last tile may end early); the first m + 1 tiles may be in
        // any order among themselves -- a stream's open hits before its chunk
        if (j + 1 < nt && j - t0 >= m + 1) {
            const TileInfo tn = w.tiles[j + 1];
            bad |= key_less(tn.base, tn.min_idx, tj.base, tj.min_idx);
        }
        if (j + m + 1 < nt) {
            const TileInfo tf = w.tiles[j + m + 1];
            bad |= !key_less(tj.max_toa, tj.max_idx, tf.base, tf.min_idx);
        }
        if (bad) atomicOr(&w.status->sort_fallback, 1);
    }

    const int64_t base = jr.start;
    const int r0 = t * IPT;
    const int first_tile = j - m < t0 ? t0 : j - m;
    const int last_tile = j + m >= nt ? nt - 1 : j + m;
    uint32_t rank[IPT];
#pragma unroll
    for (int q = 0; q < IPT; q++) rank[q] = (uint32_t)((int64_t)(first_tile - t0) * T + r0 + q);
    __shared__ uint32_t ak[IPT >= 8 ? T : 1];  // this tile's keys (merge path)
    // a neighbour tile that does not overlap this one in ToA counts all or none
    auto disjoint = [&](int i, const TileInfo& ti) {
        if (!(i < j ? tj.base >= ti.max_toa : tj.max_toa < ti.base)) return false;
        if (i < j) {
#pragma unroll
            for (int q = 0; q < IPT; q++) rank[q] += (uint32_t)ti.count;
        }
        return true;
    };
    if constexpr (IPT >= 8) {
        // Merge path of this tile (A) with each overlapping neighbour (B): a
        // neighbour element goes first when its ToA is <= (earlier tile,
        // smaller indices) or < (later tile) the element's.  Each thread
        // takes an equal share of the merged sequence: one binary search for
        // where its share starts, then a sequential merge that records, for
        // every A element it places, how many B elements precede it.
        __shared__ __align__(16) uint16_t below[T];  // per element of this tile: neighbour elements below it
        for (int e = t; e < tj.count; e += kSortThreads) ak[merge_swz(e)] = w.ts_rel[base + e];
        for (int i = first_tile; i <= last_tile; i++) {
            if (i == j) continue;
            const TileInfo ti = w.tiles[i];
            if (disjoint(i, ti)) continue;
            const bool earlier = i < j;
            // only the parts of the neighbour that can interleave with this
            // tile: parts whose last key goes before this tile's first key go
            // before all of it; parts after the first one whose last key does
            // not go before this tile's last key go before none of it
            int b0, b1;
            {
                const int S = (ti.count + kTileQ - 1) / kTileQ;
                int c_lo = 0, c_hi = 0;
#pragma unroll
                for (int k = 0; k < kTileQ; k++) {
                    const uint64_t qk = ti.base + w.tile_q[(int64_t)i * kTileQ + k];
                    c_lo += (earlier ? qk <= tj.base : qk < tj.base) ? 1 : 0;
                    c_hi += (earlier ? qk <= tj.max_toa : qk < tj.max_toa) ? 1 : 0;
                }
                b0 = c_lo * S < ti.count ? c_lo * S : ti.count;
                b1 = (c_hi + 1) * S < ti.count ? (c_hi + 1) * S : ti.count;
                if (b1 < b0) b1 = b0;
            }
            const int64_t ibase = jr.seg_start + (int64_t)(i - t0) * T + b0;
#pragma unroll
            for (int q = 0; q < IPT; q++) rank[q] += (uint32_t)b0;
            if (b1 == b0) continue;
            __syncthreads();  // nk and below of the previous neighbour are no longer read
            for (int e = t; e < b1 - b0; e += kSortThreads) nk[merge_swz(e)] = w.ts_rel[ibase + e];
            __syncthreads();
            const int na = tj.count, nb = b1 - b0;
            auto b_first = [&](int bi, int ai) {
                const uint64_t tb = ti.base + nk[merge_swz(bi)], ta = tj.base + ak[merge_swz(ai)];
                return earlier ? tb <= ta : tb < ta;
            };
            const int total = na + nb;
            const int per = (total + kSortThreads - 1) / kSortThreads;
            const int d0 = t * per < total ? t * per : total;
            const int d1 = d0 + per < total ? d0 + per : total;
            int lo = d0 - nb > 0 ? d0 - nb : 0, hi = d0 < na ? d0 : na;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (!b_first(d0 - mid - 1, mid)) lo = mid + 1; else hi = mid;
            }
            int ai = lo, bi = d0 - lo;
            for (int d = d0; d < d1; d++) {
                if (bi < nb && (ai == na || b_first(bi, ai))) {
                    bi++;
                } else {
                    below[ai] = (uint16_t)bi;
                    ai++;
                }
            }
            __syncthreads();
            // a thread's IPT counts are 16-byte aligned: read eight at a time
            // (entries past the tile's count are never used)
#pragma unroll
            for (int q = 0; q < IPT; q += 8) {
                const uint4 b = *reinterpret_cast<const uint4*>(&below[r0 + q]);
                const uint32_t bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    rank[q + 2 * k] += bw[k] & 0xFFFFu;
                    rank[q + 2 * k + 1] += bw[k] >> 16;
                }
            }
        }
    } else {
        // short tiles: a binary search per element and neighbour
        uint64_t toa[IPT];
#pragma unroll
        for (int q = 0; q < IPT; q++) toa[q] = r0 + q < tj.count ? tj.base + w.ts_rel[base + r0 + q] : ~0ull;
        for (int i = first_tile; i <= last_tile; i++) {
            if (i == j) continue;
            const TileInfo ti = w.tiles[i];
            if (disjoint(i, ti)) continue;
            const int64_t ibase = jr.seg_start + (int64_t)(i - t0) * T;
            __syncthreads();
            for (int e = t; e < ti.count; e += kSortThreads) nk[e] = w.ts_rel[ibase + e];
            __syncthreads();
            // a thread whose smallest key lies beyond the whole tile counts all of it
            const bool all = i < j ? toa[0] >= ti.max_toa : toa[0] > ti.max_toa;
            int lo = 0;
#pragma unroll
            for (int q = 0; q < IPT; q++) {
                if (r0 + q < tj.count) {
                    lo = all ? ti.count : count_below(nk, ti.count, ti.base, toa[q], i < j, lo);
                    rank[q] += (uint32_t)lo;
                }
            }
        }
    }
    // scatter: element e of the sorted tile goes to position rank(e) of its
    // chunk.  Ranks pass through LDS so that consecutive lanes take
    // consecutive elements, whose ranks are mostly consecutive too.
    __syncthreads();  // the neighbour keys are no longer read
    // four ranks per 16-byte store (entries past the tile's count are never read)
#pragma unroll
    for (int q = 0; q < IPT; q += 4)
        *reinterpret_cast<uint4*>(&nk[r0 + q]) = make_uint4(rank[q], rank[q + 1], rank[q + 2], rank[q + 3]);
    __syncthreads();
    for (int e = t; e < tj.count; e += kSortThreads) {
        const int64_t dst = jr.seg_start + nk[e];
        const uint2 pay = w.ts_pay[base + e];
        w.s_toa[dst] = tj.base + (IPT >= 8 ? ak[merge_swz(e)] : w.ts_rel[base + e]);
        w.s_idx[dst] = (int32_t)(base + (pay.x & 0xFFFFu));
        w.s_tot[dst] = (uint16_t)(pay.x >> 16);
        w.s_xy[dst] = pay.y;
    }
}

hipError_t launch_tile_merge(const Work& w, hipStream_t s)
{
    dim3 grid(xcd_grid(w.n_sort_tiles)), block(kSortThreads);
    TimedLaunch tl("tile_rank", s);
    switch (w.sort_ipt) {
    case 4: hipLaunchKernelGGL(k_tile_rank<4>, grid, block, 0, s, w); break;
    case 8: hipLaunchKernelGGL(k_tile_rank<8>, grid, block, 0, s, w); break;
    case 16: hipLaunchKernelGGL(k_tile_rank<16>, grid, block, 0, s, w); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------ sort fallback
// Sort key of the fallback: the ToA, or -- for a batch of chunks -- the chunk
// id above the ToA relative to the chunk's minimum, so chunks stay apart and
// in order.  Ties keep input order (the sort is stable), i.e. (toa, index).
struct ToaSortJob {
    static constexpr bool kKeepSorted = false;
    const hc_hit* hits;
    Work w;
    __device__ int64_t count() const { return w.n; }
    __device__ int seg_of(int64_t i) const
    {
        int a = 0, b = w.n_seg - 1;
        while (a < b) {
            const int m = (a + b + 1) >> 1;
            if (w.segs[m].start <= i) a = m; else b = m - 1;
        }
        return a;
    }
    __device__ void load(int64_t i, uint64_t& k, uint32_t& v) const
    {
        const uint64_t toa = hits[i].toa;
        v = (uint32_t)i;
        if (w.n_seg <= 1) {
            k = toa;
        } else {
            const int sg = seg_of(i);
            k = ((uint64_t)sg << w.status->rs[0].shift) | (toa - w.segs[sg].toa_min);
        }
    }
    __device__ int plan(RadixState& st, RadixLds& L)
    {
        __shared__ uint64_t red[kFbThreads / kWave];
        if (w.n_seg > 1) {  // every chunk's smallest ToA: the minimum of its tiles' minima
            for (int sg = threadIdx.x; sg < w.n_seg; sg += kFbThreads) {
                const SegInfo& si = w.segs[sg];
                const int t0 = si.tile0[kSortKind];
                const int t1 = t0 + (si.count + w.sort_tile - 1) / w.sort_tile;
                uint64_t m = ~0ull;
                for (int i = t0; i < t1; i++) m = w.tiles[i].base < m ? w.tiles[i].base : m;
                w.segs[sg].toa_min = m;
            }
            __threadfence_block();
            __syncthreads();
        }
        uint64_t mn = ~0ull, mx = 0;
        for (int i = threadIdx.x; i < w.n_sort_tiles; i += kFbThreads) {
            const TileInfo ti = w.tiles[i];
            if (w.n_seg <= 1) {
                mn = ti.base < mn ? ti.base : mn;
                mx = ti.max_toa > mx ? ti.max_toa : mx;
            } else {  // largest span of a chunk
                const uint64_t span = ti.max_toa - w.segs[w.tile_seg[kSortKind][i]].toa_min;
                mx = span > mx ? span : mx;
            }
        }
        mn = block_min_u64<kFbThreads>(mn, red);
        mx = block_max_u64<kFbThreads>(mx, red);
        if (threadIdx.x == 0) {
            bool on = w.status->sort_fallback != 0 && w.status->err_range == 0;
            uint64_t range;
            if (w.n_seg <= 1) {
                st.key_min = mn;
                range = mx - mn;
                st.shift = 0;
            } else {
                const int sb = 32 - __builtin_clz((uint32_t)(w.n_seg - 1));
                const int tb = mx == 0 ? 0 : 64 - __builtin_clzll(mx);
                if (sb + tb > 64) {  // the chunk field does not fit beside the span:
                    atomicOr(&w.status->err_span, 1);  // nothing is sorted, so every
                    atomicOr(&w.status->err_range, 1);  // later stage must stand down
                    on = false;
                }
                st.key_min = 0;
                st.shift = tb;
                range = ((uint64_t)(w.n_seg - 1) << tb) | mx;
            }
            st.active = on ? 1 : 0;
            const int bits = range == 0 ? 0 : 64 - __builtin_clzll(range);
            st.passes = bits <= 8 ? 1 : (bits + 7) / 8;
        }
        (void)L;
        return 0;
    }
    __device__ void store(int64_t pos, uint64_t rel, uint32_t v) const
    {
        const hc_hit h = hits[v];
        w.s_toa[pos] = h.toa;
        w.s_idx[pos] = (int32_t)v;
        w.s_xy[pos] = (uint32_t)h.x | ((uint32_t)h.y << 16);
        w.s_tot[pos] = h.tot;
        (void)rel;
    }
    __device__ void extra(int, const uint64_t*, const uint32_t*, RadixLds&) {}
};

__global__ __launch_bounds__(kFbThreads) void k_sort_fallback(const hc_hit* __restrict__ hits, Work w)
{
    resolve_count(w);
    if (!w.status->sort_fallback || w.status->err_range) return;  // the common case
    ToaSortJob job{hits, w};
    uint64_t* kb[2] = {w.fb_key[0], w.fb_key[1]};
    uint32_t* vb[2] = {w.fb_val[0], w.fb_val[1]};
    radix_engine(job, &w.status->rs[0], kb, vb, w.fb_hist, w.n_fb_blocks, &w.status->err_internal);
}



hipError_t launch_sort_fallback(const hc_hit* hits, const Work& w, hipStream_t s)
{
    TimedLaunch tl("sort_fallback", s);
    hipLaunchKernelGGL(k_sort_fallback, dim3(persistent_grid()), dim3(kFbThreads), 0, s, hits, w);
    return hipGetLastError();
}

}  // namespace hc
