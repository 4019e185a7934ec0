// Device-side building blocks shared by the kernels of the hit-clustering
// library: work-group scans and LDS radix sorting, XCD-aware tile mapping,
// union-find primitives and the ordering keys of the hit stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc_internal.h"

namespace hc {

constexpr int kWave = 64;

// ------------------------------------------------------------ tile mapping
// Work-groups are dispatched round-robin over the 8 XCDs of an MI355X (one
// L2 each).  Give every XCD a contiguous range of tiles, so a tile and its
// neighbours -- which read each other's data -- share an L2.
__host__ __device__ inline int xcd_grid(int ntiles) { return 8 * ((ntiles + 7) / 8); }
// The grid may be larger than xcd_grid(ntiles) (sized for a capacity while
// the tile count is read on the device): work-groups past each XCD's range
// get no tile, so no tile is taken twice.
__device__ inline int xcd_tile(int ntiles, int xcd_map = 1)
{
    const int b = blockIdx.x;
    if (!xcd_map) return b < ntiles ? b : -1;
    const int per = (ntiles + 7) / 8;
    if ((b >> 3) >= per) return -1;
    const int t = (b & 7) * per + (b >> 3);
    return t < ntiles ? t : -1;
}

// -------------------------------------------------------- tile ranges
// Hits [start, start + count) of tile `tile` of a kind with `size` hits per
// tile; seg_start / seg_end bound the chunk the tile belongs to.
struct TileRange {
    int seg;
    int count;
    int64_t start;
    int64_t seg_start, seg_end;
    int tile0, tile1;  // the chunk's tiles of this kind: [tile0, tile1)
};

__device__ inline TileRange tile_range(const Work& w, int kind, int tile, int size)
{
    TileRange r;
    if (w.n_seg <= 1) {
        r.seg = 0;
        r.seg_start = 0;
        r.seg_end = w.n;
        r.tile0 = 0;
        r.tile1 = (int)((w.n + size - 1) / size);
        r.start = (int64_t)tile * size;
    } else {
        r.seg = w.tile_seg[kind][tile];
        const SegInfo& s = w.segs[r.seg];
        r.seg_start = s.start;
        r.seg_end = s.start + s.count;
        r.tile0 = s.tile0[kind];
        r.tile1 = s.tile0[kind] + (s.count + size - 1) / size;
        r.start = s.start + (int64_t)(tile - s.tile0[kind]) * size;
    }
    const int64_t left = r.seg_end - r.start;
    r.count = (int)(left < size ? left : size);
    return r;
}

// Kernel prologue: with a device-resident hit count, replace the capacity
// bound by the actual count and derive every tile count from it.  Tiles
// beyond the count see tile_range / xcd_tile report them absent.
__device__ inline void resolve_count(Work& w)
{
    if (!w.n_dev) return;
    int32_t n = *w.n_dev;
    if (n < 0 || n > w.n) {  // never larger than the capacity the grids were sized for
        atomicOr(&w.status->err_internal, 1);
        n = 0;
    }
    w.n = n;
    w.n_sort_tiles = (n + w.sort_tile - 1) / w.sort_tile;
    w.n_link_tiles = (n + kLinkTile - 1) / kLinkTile;
    w.n_feat_tiles = (n + kFeatTile - 1) / kFeatTile;
    w.n_scan_blocks = (n + kScanBlock - 1) / kScanBlock;
    w.n_fb_blocks = (n + kFbBlock - 1) / kFbBlock;
}

__device__ inline uint64_t seg_dt(const Work& w, int seg) { return w.n_seg <= 1 ? w.dt : w.segs[seg].dt; }

// ------------------------------------------------------- saturating math
__device__ inline uint64_t sat_sub_u64(uint64_t a, uint64_t b) { return a > b ? a - b : 0; }

// (toa, input index) order: the total order the sweep of Section 4.1 uses.
__device__ inline bool key_less(uint64_t ta, int32_t ia, uint64_t tb, int32_t ib)
{
    return ta < tb || (ta == tb && ia < ib);
}

// ---------------------------------------------------------------- scans
// Exclusive scan of one value per thread across a work-group of NT threads.
// wsum: LDS scratch of NT/64 words.  *total (optional) receives the sum.
template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total)
{
    static_assert(NT % kWave == 0 && NT / kWave <= kWave, "work-group size");
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
        uint32_t s = lane < NT / kWave ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            uint32_t y = __shfl_up(s, o, kWave);
            if (lane >= o) s += y;
        }
        if (lane < NT / kWave) wsum[lane] = s;
    }
    __syncthreads();
    const uint32_t before = wid ? wsum[wid - 1] : 0u;
    if (total) *total = wsum[NT / kWave - 1];
    __syncthreads();
    return before + x - v;
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves (no LDS
// traffic): shifts of 1, 2, 4, 8 inside each row of 16 lanes, then the last
// lane of row 0 / row 2 is added to rows 1 / 3, then lane 31 to rows 2 and 3.
// Sources outside a row or disabled rows contribute 0.
__device__ inline uint32_t wave_incl_scan_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

template <int CTRL, int ROW_MASK>
__device__ inline uint64_t dpp_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROW_MASK, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROW_MASK, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_incl_scan_u64(uint64_t v)
{
    v += dpp_u64<0x111, 0xF>(v);
    v += dpp_u64<0x112, 0xF>(v);
    v += dpp_u64<0x114, 0xF>(v);
    v += dpp_u64<0x118, 0xF>(v);
    v += dpp_u64<0x142, 0xA>(v);
    v += dpp_u64<0x143, 0xC>(v);
    return v;
}

// Work-group reductions of 64-bit minima / maxima (result valid in all threads).
template <int NT>
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t* red)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(v, o, kWave);
        v = y < v ? y : v;
    }
    if (lane == 0) red[wid] = v;
    __syncthreads();
    uint64_t r = red[0];
    for (int i = 1; i < NT / kWave; i++) r = red[i] < r ? red[i] : r;
    __syncthreads();
    return r;
}

template <int NT>
__device__ inline uint64_t block_max_u64(uint64_t v, uint64_t* red)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(v, o, kWave);
        v = y > v ? y : v;
    }
    if (lane == 0) red[wid] = v;
    __syncthreads();
    uint64_t r = red[0];
    for (int i = 1; i < NT / kWave; i++) r = red[i] > r ? red[i] : r;
    __syncthreads();
    return r;
}

// ------------------------------------------------------ LDS radix sort
// Stable LSD sort of NT*IPT (u32 key, u16 value) pairs held in LDS buffers
// (k0, v0) by the low `bits` bits of the key, four bits per pass.  Thread t
// owns positions [t*IPT, (t+1)*IPT).  (k1, v1) is the second buffer; cnt
// holds 16*NT u16 counters and wsum NT/64 words.  Returns which buffer
// (0 or 1) holds the result.
template <int NT, int IPT>
__device__ inline int block_radix_sort(uint32_t* k0, uint16_t* v0, uint32_t* k1, uint16_t* v1,
                                       uint16_t* cnt, uint32_t* wsum, int bits)
{
    static_assert(IPT <= 255, "per-thread counters are bytes");
    const int t = threadIdx.x;
    int cur = 0;
    for (int shift = 0; shift < bits; shift += 4) {
        uint32_t* ki = cur ? k1 : k0;
        uint16_t* vi = cur ? v1 : v0;
        uint32_t* ko = cur ? k0 : k1;
        uint16_t* vo = cur ? v0 : v1;
        uint32_t k[IPT];
        uint16_t v[IPT];
        uint32_t d[IPT], lr[IPT];
        uint32_t c[4] = {0u, 0u, 0u, 0u};  // 16 byte-sized digit counters
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            k[j] = ki[t * IPT + j];
            v[j] = vi[t * IPT + j];
            d[j] = (k[j] >> shift) & 15u;
            const uint32_t sh = (d[j] & 3u) * 8u;
            const uint32_t r = d[j] >> 2;
            uint32_t cur_c = r == 0 ? c[0] : r == 1 ? c[1] : r == 2 ? c[2] : c[3];
            lr[j] = (cur_c >> sh) & 0xFFu;
            const uint32_t inc = 1u << sh;
            c[0] += r == 0 ? inc : 0u;
            c[1] += r == 1 ? inc : 0u;
            c[2] += r == 2 ? inc : 0u;
            c[3] += r == 3 ? inc : 0u;
        }
#pragma unroll
        for (int dd = 0; dd < 16; dd++) cnt[dd * NT + t] = (uint16_t)((c[dd >> 2] >> ((dd & 3) * 8)) & 0xFFu);
        __syncthreads();
        // exclusive scan over cnt in (digit, thread) order; thread t owns 16
        // consecutive counters
        uint32_t loc[16];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            loc[i] = cnt[t * 16 + i];
            s += loc[i];
        }
        uint32_t run = block_exclusive_scan<NT>(s, wsum, nullptr);
#pragma unroll
        for (int i = 0; i < 16; i++) {
            cnt[t * 16 + i] = (uint16_t)run;
            run += loc[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            const uint32_t dst = (uint32_t)cnt[d[j] * NT + t] + lr[j];
            ko[dst] = k[j];
            vo[dst] = v[j];
        }
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

// Stable LSD sort of the NT*IPT element indices in e0 by key[e] (the keys
// stay in place in LDS and are read through the index), the low `bits` bits,
// four bits per pass.  Half the LDS of sorting (key, index) pairs, which lets
// more work-groups share a CU.  Thread t owns positions [t*IPT, (t+1)*IPT);
// e1 is the second buffer, cnt holds 16*NT u16 counters and wsum NT/64
// words.  Returns which buffer (0 or 1) holds the sorted indices.
template <int NT, int IPT>
__device__ inline int block_radix_sort_index(const uint32_t* key, uint16_t* e0, uint16_t* e1, uint16_t* cnt,
                                             uint32_t* wsum, int bits)
{
    static_assert(IPT <= 255, "per-thread counters are bytes");
    const int t = threadIdx.x;
    int cur = 0;
    for (int shift = 0; shift < bits; shift += 4) {
        uint16_t* ei = cur ? e1 : e0;
        uint16_t* eo = cur ? e0 : e1;
        uint16_t e[IPT];
        uint32_t dl[IPT];  // digit | rank among the thread's equal digits << 4
        uint32_t c[4] = {0u, 0u, 0u, 0u};  // 16 byte-sized digit counters
#pragma unroll
        for (int j = 0; j < IPT; j++) e[j] = ei[t * IPT + j];
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            const uint32_t d = (key[e[j]] >> shift) & 15u;
            const uint32_t sh = (d & 3u) * 8u;
            const uint32_t r = d >> 2;
            const uint32_t cur_c = r == 0 ? c[0] : r == 1 ? c[1] : r == 2 ? c[2] : c[3];
            dl[j] = d | (((cur_c >> sh) & 0xFFu) << 4);
            const uint32_t inc = 1u << sh;
            c[0] += r == 0 ? inc : 0u;
            c[1] += r == 1 ? inc : 0u;
            c[2] += r == 2 ? inc : 0u;
            c[3] += r == 3 ? inc : 0u;
        }
#pragma unroll
        for (int dd = 0; dd < 16; dd++) cnt[dd * NT + t] = (uint16_t)((c[dd >> 2] >> ((dd & 3) * 8)) & 0xFFu);
        __syncthreads();
        // exclusive scan over cnt in (digit, thread) order; thread t owns 16
        // consecutive counters (read twice rather than held in registers)
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < 16; i++) sum += cnt[t * 16 + i];
        uint32_t run = block_exclusive_scan<NT>(sum, wsum, nullptr);
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const uint32_t v = cnt[t * 16 + i];
            cnt[t * 16 + i] = (uint16_t)run;
            run += v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++) eo[(uint32_t)cnt[(dl[j] & 15u) * NT + t] + (dl[j] >> 4)] = e[j];
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

// Rank of cluster root `root` (an input index of chunk `seg`, which starts at
// input index seg_start) in ascending label order over all chunks: the roots
// of earlier blocks (blk_off), of earlier mask words of its block
// (root_wpre) and below it in its word.  Valid once the flatten pass and the
// block scan have run.
__device__ inline uint32_t root_rank(const Work& w, int seg, int64_t seg_start, int32_t root)
{
    const int64_t o = (int64_t)root - seg_start;
    const int64_t b = (w.n_seg > 1 ? w.segs[seg].tile0[kScanKind] : 0) + o / kScanBlock;
    const int bit = (int)(o % kScanBlock);
    const int64_t wd = b * (kScanBlock / 64) + bit / 64;
    const unsigned long long below = (1ull << (bit % 64)) - 1ull;
    return w.blk_off[b] + w.root_wpre[wd] + (uint32_t)__popcll(w.root_mask[wd] & below);
}

// ------------------------------------------------------- spin waiting
__device__ inline int32_t ld_acquire(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (whole work-group) until *p >= target.  Only ever used on counters
// advanced by tasks holding smaller tickets, so every wait ends.
__device__ inline void wait_at_least(const int32_t* p, int32_t target, int32_t* lds_flag)
{
    if (threadIdx.x == 0) {
        // back off: hundreds of waiting work-groups polling one counter at a
        // high rate would crowd out the memory traffic of the task they wait for
        int spins = 0;
        while (ld_acquire(p) < target) {
            if (spins < 16) {
                __builtin_amdgcn_s_sleep(8);
                spins++;
            } else {
                __builtin_amdgcn_s_sleep(127);
            }
        }
    }
    __syncthreads();
    __threadfence();
    (void)lds_flag;
}

__device__ inline void signal_done(int32_t* p)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(p, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------- union-find (global)
// Forest over input indices; parent[i] <= i always, the root of a tree is
// its smallest index (the canonical label).  Path halving; links the larger
// root under the smaller with compare-and-swap.  Concurrent halving stores
// only ever install ancestors, so races are benign.
// Every pointer satisfies 0 <= parent[x] <= x; a value outside that range
// can only come from an internal inconsistency, which is flagged in *err and
// treated as a root so that no access leaves the array.
__device__ inline int32_t gfind(int32_t* parent, int32_t x, int32_t* err)
{
    while (true) {
        int32_t p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        if (p < 0 || p > x) {
            atomicOr(err, 1);
            return x;
        }
        int32_t g = __hip_atomic_load(parent + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (g < 0 || g > p) {
            atomicOr(err, 1);
            return p;
        }
        if (g != p) __hip_atomic_store(parent + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = g;
    }
}

// Root of x once no union runs any more (after the last kernel that links):
// plain, cacheable loads, and no path writes.  Every value read is an
// ancestor, so the walk ends at the root.
__device__ inline int32_t gfind_final(const int32_t* __restrict__ parent, int32_t x, int32_t* err)
{
    while (true) {
        const int32_t p = parent[x];
        if (p == x) return x;
        if (p < 0 || p > x) {
            atomicOr(err, 1);
            return x;
        }
        x = p;
    }
}

__device__ inline void gunion(int32_t* parent, int32_t a, int32_t b, int32_t* err)
{
    while (true) {
        a = gfind(parent, a, err);
        b = gfind(parent, b, err);
        if (a == b) return;
        if (a > b) {
            int32_t t = a;
            a = b;
            b = t;
        }
        int32_t expected = b;
        if (__hip_atomic_compare_exchange_strong(parent + b, &expected, a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        b = expected;
    }
}

}  // namespace hc
