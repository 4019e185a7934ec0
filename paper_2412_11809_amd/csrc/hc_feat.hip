// Step A4 of the clustering path: per-cluster features and the output table.
//
// The paper's pipeline ends by sorting clusters by their first ToA (Step 6 of
// its high-level GPU algorithm) and names feature extraction as the next GPU
// task (Section 6).  Here the features are reduced without moving any hit:
//   k_features  per tile of kFeatTile sorted hits: an LDS hash keyed by the
//               cluster label gathers each cluster's partial sums (size, ToT,
//               x*ToT, y*ToT, x, y) and ToA min/max with LDS atomics.  The one
//               tile that holds the cluster's label hit (idx == label) stores
//               its partial as the cluster's record; every other tile queues
//               its partial as a "carry";
//   k_carries   folds the carries into the records with 64-bit atomics;
//   k_compact   decoupled look-back scan over input indices: every index with
//               labels[i] == i is a cluster, and its record becomes
//               features[rank] (ascending label order) with the centroid
//               cx = (double)sum_x_tot / (double)sum_tot (IEEE division).
#include "hc_device.h"

namespace hc {

__device__ inline uint32_t root_hash(uint32_t key) { return (key * 0x9E3779B1u) >> 22; }  // 10 bits

__global__ __launch_bounds__(kFeatThreads) void k_features(Work w, const int32_t* __restrict__ labels)
{
    static_assert(kFeatHash == 1024, "root_hash yields 10 bits");
    __shared__ uint32_t h_key[kFeatHash];
    __shared__ uint32_t a_size[kFeatHash], a_st[kFeatHash], a_sx[kFeatHash], a_sy[kFeatHash], a_own[kFeatHash];
    __shared__ unsigned long long a_sxt[kFeatHash], a_syt[kFeatHash], a_tmin[kFeatHash], a_tmax[kFeatHash];
    constexpr int PER = kFeatTile / kFeatThreads;

    if (w.status->err_range) return;
    const int tile = xcd_tile(w.n_feat_tiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)tile * kFeatTile;
    for (int i = t; i < kFeatHash; i += kFeatThreads) h_key[i] = 0u;
    __syncthreads();

    int slot[PER];
    int32_t idx[PER];
    uint64_t toa[PER];
    uint32_t xy[PER], tot[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t p = p0 + t + q * kFeatThreads;
        slot[q] = -1;
        if (p < w.n) {
            idx[q] = w.s_idx[p];
            toa[q] = w.s_toa[p];
            xy[q] = w.s_xy[p];
            tot[q] = w.s_tot[p];
            int32_t lab = 0;
            if (idx[q] >= 0 && idx[q] < w.n) lab = labels[idx[q]];
            else atomicOr(&w.status->err_internal, 1);
            if (lab < 0 || lab >= w.n) {
                atomicOr(&w.status->err_internal, 1);
                lab = 0;
            }
            const uint32_t key = (uint32_t)lab + 1u;
            uint32_t s = root_hash(key);
            while (true) {
                const uint32_t old = atomicCAS(&h_key[s], 0u, key);
                if (old == 0u) {  // first hit of this cluster here: initialise
                    a_size[s] = 0u;
                    a_st[s] = 0u;
                    a_sx[s] = 0u;
                    a_sy[s] = 0u;
                    a_own[s] = 0u;
                    a_sxt[s] = 0ull;
                    a_syt[s] = 0ull;
                    a_tmin[s] = ~0ull;
                    a_tmax[s] = 0ull;
                    break;
                }
                if (old == key) break;
                s = (s + 1u) & (kFeatHash - 1);
            }
            slot[q] = (int)s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int s = slot[q];
        if (s < 0) continue;
        const uint32_t x = xy[q] & 0xFFFFu, y = xy[q] >> 16;
        atomicAdd(&a_size[s], 1u);
        atomicAdd(&a_st[s], tot[q]);
        atomicAdd(&a_sx[s], x);
        atomicAdd(&a_sy[s], y);
        atomicAdd(&a_sxt[s], (unsigned long long)x * tot[q]);
        atomicAdd(&a_syt[s], (unsigned long long)y * tot[q]);
        atomicMin(&a_tmin[s], (unsigned long long)toa[q]);
        atomicMax(&a_tmax[s], (unsigned long long)toa[q]);
        if ((uint32_t)idx[q] + 1u == h_key[s]) a_own[s] = 1u;
    }
    __syncthreads();
    for (int s = t; s < kFeatHash; s += kFeatThreads) {
        const uint32_t key = h_key[s];
        if (key == 0u) continue;
        SlotRec r;
        r.size = a_size[s];
        r.root = (int32_t)(key - 1u);
        r.sum_tot = a_st[s];
        r.toa_min = a_tmin[s];
        r.toa_max = a_tmax[s];
        r.sum_xt = a_sxt[s];
        r.sum_yt = a_syt[s];
        r.sum_x = a_sx[s];
        r.sum_y = a_sy[s];
        if (a_own[s]) {
            w.slots[key - 1u] = r;
        } else {
            const int c = atomicAdd(&w.status->n_carries, 1);
            if (c < w.carry_cap) w.carries[c] = r;
            else atomicOr(&w.status->err_internal, 1);
        }
    }
}

hipError_t launch_features(const Work& w, const int32_t* labels, hipStream_t s)
{
    TimedLaunch tl("features", s);
    hipLaunchKernelGGL(k_features, dim3(xcd_grid(w.n_feat_tiles)), dim3(kFeatThreads), 0, s, w, labels);
    return hipGetLastError();
}

__global__ void k_carries(Work w)
{
    if (w.status->err_range) return;
    const int64_t nc = w.status->n_carries < w.carry_cap ? w.status->n_carries : w.carry_cap;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        const SlotRec r = w.carries[c];
        if (r.root < 0 || r.root >= w.n) {
            atomicOr(&w.status->err_internal, 1);
            continue;
        }
        SlotRec* d = w.slots + r.root;
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

hipError_t launch_carries(const Work& w, hipStream_t s)
{
    TimedLaunch tl("carries", s);
    hipLaunchKernelGGL(k_carries, dim3(256), dim3(256), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------------------ compaction
constexpr unsigned long long kAgg = 1ull << 62, kIncl = 2ull << 62, kValMask = (1ull << 62) - 1;

__global__ __launch_bounds__(kScanThreads) void k_compact(Work w, const int32_t* __restrict__ labels,
                                                          hc_features* __restrict__ out, int32_t* n_clusters)
{
    constexpr int PER = kScanBlock / kScanThreads;
    __shared__ int s_tile;
    __shared__ uint32_t wsum[kScanThreads / kWave];
    __shared__ unsigned long long s_prefix;
    const int t = threadIdx.x;
    if (t == 0) s_tile = atomicAdd(&w.status->scan_ticket, 1);
    __syncthreads();
    const int tile = s_tile;
    if (w.status->err_range || w.status->err_internal) {
        if (tile == 0 && t == 0) *n_clusters = w.status->err_range ? HC_ERR_RANGE : HC_ERR_DEVICE;
        return;
    }
    const int64_t i0 = (int64_t)tile * kScanBlock + (int64_t)t * PER;
    uint32_t flags = 0, c = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t i = i0 + q;
        if (i < w.n && labels[i] == (int32_t)i) {
            flags |= 1u << q;
            c++;
        }
    }
    uint32_t total;
    const uint32_t off = block_exclusive_scan<kScanThreads>(c, wsum, &total);
    if (t == 0) {
        unsigned long long prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(&w.scan_state[0], kIncl | total, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&w.scan_state[tile], kAgg | total, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            int pred = tile - 1;
            while (true) {
                unsigned long long v;
                while ((v = __hip_atomic_load(&w.scan_state[pred], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) == 0ull)
                    __builtin_amdgcn_s_sleep(1);
                prefix += v & kValMask;
                if (v & kIncl) break;
                pred--;
            }
            __hip_atomic_store(&w.scan_state[tile], kIncl | (prefix + total), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_prefix = prefix;
        if (tile == w.n_scan_blocks - 1) *n_clusters = (int32_t)(prefix + total);
    }
    __syncthreads();
    if (!out) return;
    uint64_t k = s_prefix + off;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        if (!(flags & (1u << q))) continue;
        const int64_t i = i0 + q;
        const SlotRec r = w.slots[i];
        hc_features f;
        f.label = (int32_t)i;
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
        out[k++] = f;
    }
}

hipError_t launch_compact(const Work& w, const int32_t* labels, hc_features* features, int32_t* n_clusters,
                          hipStream_t s)
{
    TimedLaunch tl("compact", s);
    hipLaunchKernelGGL(k_compact, dim3(w.n_scan_blocks), dim3(kScanThreads), 0, s, w, labels, features, n_clusters);
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
