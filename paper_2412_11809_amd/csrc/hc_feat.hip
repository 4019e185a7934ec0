// Step A4 of the clustering path: per-cluster features and the output table.
//
// The paper's pipeline ends by sorting clusters by their first ToA (Step 6 of
// its high-level GPU algorithm) and names feature extraction as the next GPU
// task (Section 6).  Here the features are reduced without moving any hit:
//   k_features  per tile of kFeatTile sorted hits: an LDS hash keyed by the
//               cluster label gathers each cluster's partial sums (size, ToT,
//               x*ToT, y*ToT, and x, y where a ToT is zero) and its ToA
//               min/max (32-bit offsets from the tile's first ToA; in the
//               rare tile whose ToA span exceeds 32 bits, the tile positions
//               of the cluster's first and last hit, the tile being in ToA
//               order) with LDS atomics.  The one tile that holds the
//               cluster's label hit (idx == label) stores its partial as the
//               cluster's record, at the cluster's rank in ascending label
//               order; every other tile queues its partial as a "carry";
//   k_scan_blocks  (runs before k_features) the flatten pass flagged every
//               root (labels[i] == i) in a bit mask, with counts per block
//               of input indices and per mask word; one work-group scans the
//               block counts, which makes every root's rank three loads away;
//   k_carries   folds the carries into the records with 64-bit atomics;
//   k_compact   streams the rank-ordered records into features[rank] with
//               the centroid cx = (double)sum_x_tot / (double)sum_tot (IEEE
//               division).
#include "hc_device.h"

namespace hc {

__device__ inline uint32_t root_hash(uint32_t key) { return (key * 0x9E3779B1u) >> 23; }  // 9 bits

__global__ __launch_bounds__(kFeatThreads) void k_features(Work w, const int32_t* __restrict__ labels)
{
    resolve_count(w);
    static_assert(kFeatHash == 512 && kFeatHash >= kFeatTile, "root_hash yields 9 bits; a tile never fills the table");
    static_assert((uint64_t)kFeatTile * 65535u < (1ull << 32), "paired 32-bit sums must not carry");
    // label + 1 (below 2^31), bit 31 set once the cluster's label hit is seen
    __shared__ uint32_t h_key[kFeatHash];
    // two 32-bit sums per 64-bit word (size | sum ToT << 32, sum x | sum y << 32):
    // a tile's sums stay below 2^32, so one atomic adds both without carry
    __shared__ unsigned long long a_cs[kFeatHash], a_xy[kFeatHash];
    __shared__ unsigned long long a_sxt[kFeatHash], a_syt[kFeatHash];
    // ToA min / max: offsets from the tile's first ToA, or tile positions in a wide tile
    __shared__ uint32_t a_pmin[kFeatHash], a_pmax[kFeatHash];
    constexpr uint32_t kOwn = 0x80000000u;
    constexpr int PER = kFeatTile / kFeatThreads;

    if (w.status->err_range) return;
    const int tile = xcd_tile(w.n_feat_tiles, w.xcd_map);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const TileRange tr = tile_range(w, kFeatKind, tile, kFeatTile);
    const int64_t p0 = tr.start;
    const int64_t p_end = tr.start + tr.count;
    const int32_t lab0 = w.n_seg > 1 ? (int32_t)tr.seg_start : 0;  // labels are chunk-local in a batch
    for (int i = t; i < kFeatHash; i += kFeatThreads) h_key[i] = 0u;
    const uint64_t tfirst = p_end > p0 ? w.s_toa[p0] : 0ull;
    const bool wide = p_end > p0 && w.s_toa[p_end - 1] - tfirst > 0xFFFFFFFFull;
    __syncthreads();

    int slot[PER];
    int32_t idx[PER];
    uint64_t toa[PER];
    uint32_t xy[PER], tot[PER];
    const int lane = t & (kWave - 1);
    const unsigned long long le_mask = lane == kWave - 1 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t p = p0 + t + q * kFeatThreads;
        const bool valid = p < p_end;
        toa[q] = tfirst;
        uint32_t key = 0u;  // label + 1; 0 for no hit
        if (valid) {
            // read once by this pass: streamed past the caches the gathers use
            idx[q] = __builtin_nontemporal_load(w.s_idx + p);
            toa[q] = __builtin_nontemporal_load(w.s_toa + p);
            xy[q] = __builtin_nontemporal_load(w.s_xy + p);
            tot[q] = __builtin_nontemporal_load(w.s_tot + p);
            int32_t lab = 0;
            if (idx[q] >= 0 && idx[q] < w.n) lab = labels[idx[q]] + lab0;
            else atomicOr(&w.status->err_internal, 1);
            if (lab < 0 || lab >= w.n) {
                atomicOr(&w.status->err_internal, 1);
                lab = 0;
            }
            key = (uint32_t)lab + 1u;
        }
        // only the first lane of each run of one cluster in the wave looks the
        // cluster up in the hash; the run takes its slot from that lane
        const uint32_t kp = (uint32_t)__shfl_up((int)key, 1, kWave);
        const bool head = lane == 0 || kp != key;
        const int start = kWave - 1 - __clzll(__ballot(head) & le_mask);
        int s = -1;
        if (head && valid) {
            uint32_t h = root_hash(key);
            while (true) {
                const uint32_t old = atomicCAS(&h_key[h], 0u, key);
                if (old == 0u) {  // first hit of this cluster here: initialise
                    a_cs[h] = 0ull;
                    a_xy[h] = 0ull;
                    a_sxt[h] = 0ull;
                    a_syt[h] = 0ull;
                    a_pmin[h] = ~0u;
                    a_pmax[h] = 0u;
                    break;
                }
                if (old == key) break;
                h = (h + 1u) & (kFeatHash - 1);
            }
            s = (int)h;
        }
        s = __shfl(s, start, kWave);
        slot[q] = valid ? s : -1;
    }
    __syncthreads();
    // Consecutive sorted hits of one cluster sit in consecutive lanes: reduce
    // each run of equal slots inside the wave first, so only the run's last
    // lane touches the LDS accumulators.  A run's sums are differences of
    // wave-wide prefix sums (DPP scans, no LDS), its size is its length, and
    // -- the lanes being in ToA order -- its ToA minimum is at its first lane
    // and its maximum at its last.
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int s = slot[q];
        const int sp = __shfl_up(s, 1, kWave);
        const bool head = lane == 0 || sp != s;
        const unsigned long long heads = __ballot(head);
        const int start = kWave - 1 - __clzll(heads & le_mask);
        const bool tail = lane == kWave - 1 || ((heads >> (lane + 1)) & 1ull);
        const bool valid = s >= 0;
        const uint32_t x = valid ? (xy[q] & 0xFFFFu) : 0u, y = valid ? (xy[q] >> 16) : 0u;
        const uint32_t st = valid ? tot[q] : 0u;
        const bool own_lane = valid && (uint32_t)idx[q] + 1u == (h_key[s] & ~kOwn);
        const unsigned long long owners = __ballot(own_lane);
        const uint32_t P_st = wave_incl_scan_u32(st);
        const uint64_t P_sxt = wave_incl_scan_u64((uint64_t)x * st);
        const uint64_t P_syt = wave_incl_scan_u64((uint64_t)y * st);
        // the unweighted coordinate sums only serve a cluster whose ToTs are
        // all zero; a wave without a zero ToT cannot hold a hit of one
        const bool zero_tot = __ballot(valid && st == 0u) != 0ull;
        uint32_t P_sx = 0, P_sy = 0;
        if (zero_tot) {
            P_sx = wave_incl_scan_u32(x);
            P_sy = wave_incl_scan_u32(y);
        }
        // prefix sums just before the run (lane start - 1; 0 for a run at lane
        // 0).  Every lane takes part in each shuffle: a lane that sat one out
        // would not supply its value to the lanes reading from it.
        const int src = start > 0 ? start - 1 : 0;
        const bool first = start == 0;
        const uint32_t B_st = __shfl(P_st, src, kWave);
        uint32_t B_sx = 0, B_sy = 0;
        if (zero_tot) {
            B_sx = __shfl(P_sx, src, kWave);
            B_sy = __shfl(P_sy, src, kWave);
        }
        const uint64_t B_sxt = __shfl(P_sxt, src, kWave), B_syt = __shfl(P_syt, src, kWave);
        const uint32_t pos = wide ? (uint32_t)(t + q * kFeatThreads) : (uint32_t)(toa[q] - tfirst);
        const uint32_t pmn = (uint32_t)__shfl((int)pos, start, kWave);
        if (tail && valid) {
            const unsigned long long run = le_mask & ~((1ull << start) - 1ull);
            const uint64_t n_st = P_st - (first ? 0u : B_st);
            const uint64_t n_sx = P_sx - (first ? 0u : B_sx), n_sy = P_sy - (first ? 0u : B_sy);
            atomicAdd(&a_cs[s], (unsigned long long)((uint64_t)(lane - start + 1) | (n_st << 32)));
            if (zero_tot) atomicAdd(&a_xy[s], (unsigned long long)(n_sx | (n_sy << 32)));
            atomicAdd(&a_sxt[s], (unsigned long long)(P_sxt - (first ? 0ull : B_sxt)));
            atomicAdd(&a_syt[s], (unsigned long long)(P_syt - (first ? 0ull : B_syt)));
            atomicMin(&a_pmin[s], pmn);
            atomicMax(&a_pmax[s], pos);
            if (owners & run) atomicOr(&h_key[s], kOwn);
        }
    }
    __syncthreads();
    // Records: the owner tile writes the cluster's slot; every other tile
    // queues a carry in its own region of kFeatHash entries (positions from a
    // block scan of the per-thread counts), with no global counter.
    constexpr int SPT = kFeatHash / kFeatThreads;  // hash entries per thread
    uint32_t nc = 0;
#pragma unroll
    for (int k = 0; k < SPT; k++) {
        const int s = t + k * kFeatThreads;
        nc += (h_key[s] != 0u && !(h_key[s] & kOwn)) ? 1u : 0u;
    }
    __shared__ uint32_t wsum[kFeatThreads / kWave];
    uint32_t total;
    uint32_t pos = block_exclusive_scan<kFeatThreads>(nc, wsum, &total);
    if (t == 0) w.tile_ncarry[tile] = (int32_t)total;
    const int64_t base = (int64_t)tile * kFeatHash;
#pragma unroll
    for (int k = 0; k < SPT; k++) {
        const int s = t + k * kFeatThreads;
        const uint32_t hk = h_key[s];
        if (hk == 0u) continue;
        const uint32_t key = hk & ~kOwn;
        SlotRec r;
        const uint64_t cs = a_cs[s], sxy = a_xy[s];
        r.size = (uint32_t)cs;
        r.root = (int32_t)(key - 1u);
        r.sum_tot = cs >> 32;
        r.toa_min = wide ? w.s_toa[p0 + a_pmin[s]] : tfirst + a_pmin[s];
        r.toa_max = wide ? w.s_toa[p0 + a_pmax[s]] : tfirst + a_pmax[s];
        r.sum_xt = a_sxt[s];
        r.sum_yt = a_syt[s];
        r.sum_x = (uint32_t)sxy;
        r.sum_y = sxy >> 32;
        if (hk & kOwn) {
            w.slots[root_rank(w, tr.seg, tr.seg_start, r.root)] = r;
        } else {
            w.carries[base + pos++] = r;  // pos < kFeatHash: one entry per hash slot at most
        }
    }
}

hipError_t launch_features(const Work& w, const int32_t* labels, hipStream_t s)
{
    TimedLaunch tl("features", s);
    hipLaunchKernelGGL(k_features, dim3(xcd_grid(w.n_feat_tiles)), dim3(kFeatThreads), 0, s, w, labels);
    return hipGetLastError();
}

// Folds every tile's carries into the owners' records (64-bit atomics):
// one work-group per feature tile (grid-stride), most tiles have none.
__global__ __launch_bounds__(64) void k_carries(Work w)
{
    resolve_count(w);
    if (w.status->err_range) return;
    for (int64_t k = blockIdx.x; k < w.n_feat_tiles; k += gridDim.x) {
        const int nc = w.tile_ncarry[k];
        const TileRange tr = tile_range(w, kFeatKind, (int)k, kFeatTile);
        for (int c = threadIdx.x; c < nc; c += blockDim.x) {
            const SlotRec r = w.carries[k * kFeatHash + c];
            if (r.root < tr.seg_start || r.root >= tr.seg_end) {
                atomicOr(&w.status->err_internal, 1);
                continue;
            }
            SlotRec* d = w.slots + root_rank(w, tr.seg, tr.seg_start, r.root);
            atomicAdd(&d->size, r.size);
            atomicAdd((unsigned long long*)&d->sum_tot, (unsigned long long)r.sum_tot);
            atomicAdd((unsigned long long*)&d->sum_xt, (unsigned long long)r.sum_xt);
            atomicAdd((unsigned long long*)&d->sum_yt, (unsigned long long)r.sum_yt);
            atomicAdd((unsigned long long*)&d->sum_x, (unsigned long long)r.sum_x);
            atomicAdd((unsigned long long*)&d->sum_y, (unsigned long long)r.sum_y);
            atomicMin((unsigned long long*)&d->toa_min, (unsigned long long)r.toa_min);
            atomicMax((unsigned long long*)&d->toa_max, (unsigned long long)r.toa_max);
        }
    }
}

hipError_t launch_carries(const Work& w, hipStream_t s)
{
    TimedLaunch tl("carries", s);
    const int grid = w.n_feat_tiles < 8192 ? (w.n_feat_tiles > 0 ? w.n_feat_tiles : 1) : 8192;
    hipLaunchKernelGGL(k_carries, dim3(grid), dim3(64), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------------------ compaction
// Exclusive scan of the per-block root counts (one work-group), which also
// writes the cluster count (or the error status) to the caller.
__global__ __launch_bounds__(1024) void k_scan_blocks(Work w, int32_t* n_clusters)
{
    resolve_count(w);
    __shared__ uint32_t wsum[1024 / kWave];
    const Status* st = w.status;
    if (st->err_range || st->err_internal || st->err_span) {
        const int32_t code = (st->err_range || st->err_span) ? HC_ERR_RANGE : HC_ERR_DEVICE;
        for (int sg = threadIdx.x; sg < w.n_seg; sg += blockDim.x) n_clusters[sg] = code;
        return;
    }
    uint32_t carry = 0;
    for (int c0 = 0; c0 < w.n_scan_blocks; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < w.n_scan_blocks ? w.blk_count[i] : 0u;
        uint32_t total;
        const uint32_t e = block_exclusive_scan<1024>(v, wsum, &total);
        if (i < w.n_scan_blocks) w.blk_off[i] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) w.blk_off[w.n_scan_blocks] = carry;
    if (w.n_seg <= 1) {
        if (threadIdx.x == 0) *n_clusters = (int32_t)carry;
        return;
    }
    __syncthreads();
    for (int sg = threadIdx.x; sg < w.n_seg; sg += blockDim.x) {  // clusters per chunk
        const SegInfo& si = w.segs[sg];
        const int b0 = si.tile0[kScanKind], b1 = b0 + (si.count + kScanBlock - 1) / kScanBlock;
        n_clusters[sg] = (int32_t)(w.blk_off[b1] - w.blk_off[b0]);
    }
}

// features[rank] from the rank-ordered records of the roots of one block of
// kScanBlock input indices (ranks blk_off[b] .. blk_off[b + 1] - 1).
__global__ __launch_bounds__(kScanThreads) void k_compact(Work w, hc_features* __restrict__ out)
{
    resolve_count(w);
    const Status* st = w.status;
    if (st->err_range || st->err_internal || st->err_span || (int)blockIdx.x >= w.n_scan_blocks) return;
    const int b = blockIdx.x, t = threadIdx.x;
    const TileRange tr = tile_range(w, kScanKind, b, kScanBlock);
    const uint32_t r0 = w.blk_off[b], r1 = w.blk_off[b + 1];
    const int64_t first = w.n_seg > 1 ? w.segs[tr.seg].out - (int64_t)w.blk_off[tr.tile0] : 0;
    for (uint32_t k = r0 + t; k < r1; k += kScanThreads) {
        const SlotRec r = w.slots[k];
        hc_features f;
        f.label = (int32_t)(r.root - tr.seg_start);
        f.size = r.size;
        f.sum_tot = r.sum_tot;
        f.toa_min = r.toa_min;
        f.toa_max = r.toa_max;
        f.sum_x_tot = r.sum_xt;
        f.sum_y_tot = r.sum_yt;
        if (r.sum_tot > 0) {
            f.cx = (double)r.sum_xt / (double)r.sum_tot;
            f.cy = (double)r.sum_yt / (double)r.sum_tot;
        } else {
            f.cx = (double)r.sum_x / (double)r.size;
            f.cy = (double)r.sum_y / (double)r.size;
        }
        out[first + k] = f;
    }
}

hipError_t launch_scan_blocks(const Work& w, int32_t* n_clusters, hipStream_t s)
{
    TimedLaunch tl("scan_blocks", s);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, w, n_clusters);
    return hipGetLastError();
}

hipError_t launch_compact(const Work& w, hc_features* features, hipStream_t s)
{
    TimedLaunch tl("compact", s);
    hipLaunchKernelGGL(k_compact, dim3(w.n_scan_blocks), dim3(kScanThreads), 0, s, w, features);
    return hipGetLastError();
}

__global__ void k_write_count(int32_t* p, int32_t v) { *p = v; }

hipError_t launch_write_count(int32_t* n_clusters, int32_t value, hipStream_t s)
{
    TimedLaunch tl("write_count", s);
    hipLaunchKernelGGL(k_write_count, dim3(1), dim3(1), 0, s, n_clusters, value);
    return hipGetLastError();
}

}  // namespace hc
