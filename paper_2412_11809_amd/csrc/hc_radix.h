// Ticketed LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits.
//
// Used only on fallback paths, so it is built for robustness rather than
// speed: it runs inside ONE persistent launch whose work-groups draw task
// tickets from a counter.  A task waits only for tasks with smaller tickets
// (which are already held by running work-groups), so the launch needs no
// co-residency guarantee and every wait ends.  Task 0 decides whether the
// sort is needed at all; if not, every other work-group exits at once.
//
// Tasks: 0 = plan; then per pass p: kFbBlock-sized histogram tasks, the
// digit-counter scan in segments of kFbScanSeg counters (one task each), one
// task scanning the segment totals, scatter tasks; then `extra` caller tasks
// (queries on the result).  Sorting is stable, so equal keys keep their
// source order.
#pragma once

#include "hc_device.h"

namespace hc {

struct RadixLds {
    uint32_t k0[kFbBlock], k1[kFbBlock];
    uint16_t v0[kFbBlock], v1[kFbBlock];
    uint16_t cnt[16 * kFbThreads];
    uint32_t wsum[kFbThreads / kWave];
    uint64_t key[kFbBlock];
    uint32_t val[kFbBlock];
    uint32_t hist[256];
    uint32_t start[256];
    int32_t task;
    int32_t misc;
};

// Exclusive scan of `len` u32 counters in place by one work-group.
__device__ inline void radix_scan_counts(uint32_t* h, int64_t len, RadixLds& L)
{
    constexpr int PER = 8;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < len; c0 += (int64_t)kFbThreads * PER) {
        uint32_t v[PER];
        uint32_t s = 0;
        const int64_t b = c0 + (int64_t)threadIdx.x * PER;
#pragma unroll
        for (int j = 0; j < PER; j++) {
            v[j] = (b + j < len) ? h[b + j] : 0u;
            s += v[j];
        }
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan<kFbThreads>(s, L.wsum, &total);
#pragma unroll
        for (int j = 0; j < PER; j++) {
            if (b + j < len) h[b + j] = run;
            run += v[j];
        }
        carry += total;
    }
}

// Src: int64 count() const; void load(int64 i, uint64& key, uint32& val) const
//      (pass-0 keys, raw: the engine subtracts st.key_min).
// Plan: __device__ void plan(RadixState& st, RadixLds& L) run by task 0's
//      work-group; sets st.active, st.key_min, st.passes (>= 1) and the
//      number of extra tasks through its return value.  It may also lower
//      st.n_eff (preset to count()): only elements 0..n_eff-1 are sorted.
// Final: void store(int64 pos, uint64 rel_key, uint32 val) for the last pass.
// Extra: void extra(int task, const uint64* keys, const uint32* vals, RadixLds& L)
template <class Job>
__device__ void radix_engine(Job& job, RadixState* st, uint64_t* key_buf[2], uint32_t* val_buf[2],
                             uint32_t* hist, int32_t nb_max, int32_t* err)
{
    __shared__ RadixLds L;
    const int t = threadIdx.x;
    const int64_t n_max = job.count();
    while (true) {
        __syncthreads();
        if (t == 0) L.task = __hip_atomic_fetch_add(&st->ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int task = L.task;
        if (task == 0) {
            if (t == 0) {
                st->active = 0;
                st->passes = 1;
                st->key_min = 0;
                st->total_tasks = 1;
                st->n_eff = (int32_t)n_max;
            }
            __syncthreads();
            const int extra = job.plan(*st, L);
            __syncthreads();
            if (t == 0) {
                const int nbe = (int)((st->n_eff + kFbBlock - 1) / kFbBlock);
                if (st->n_eff < 0 || st->n_eff > n_max || nbe > nb_max) {  // more than the buffers hold
                    atomicOr(err, 1);
                    st->active = 0;
                }
                const int nh = (nbe + kFbGroup - 1) / kFbGroup;
                if (st->active) st->total_tasks = 1 + st->passes * (2 * nh + fb_scan_segments(nbe) + 1) + extra;
                __threadfence();
                __hip_atomic_store(&st->plan_done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            continue;
        }
        wait_at_least(&st->plan_done, 1, nullptr);
        if (task >= __hip_atomic_load(&st->total_tasks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        const int passes = st->passes;
        const uint64_t kmin = st->key_min;
        const int64_t n = st->n_eff;  // elements sorted; the counters are laid out for nbe blocks
        const int nb = (int)((n + kFbBlock - 1) / kFbBlock);  // <= nb_max, checked by the plan
        const int nseg = fb_scan_segments(nb);
        const int nh = (nb + kFbGroup - 1) / kFbGroup;  // tasks of kFbGroup blocks
        const int per_pass = 2 * nh + nseg + 1;
        const int64_t n_counters = (int64_t)256 * nb;
        uint32_t* seg_tot = hist + n_counters;
        const int tt = task - 1;
        if (tt >= passes * per_pass) {
            wait_at_least(&st->scatter_done[passes - 1], nh, nullptr);
            const int last = (passes - 1) & 1;
            job.extra(tt - passes * per_pass, key_buf[last], val_buf[last], L);
            continue;
        }
        const int p = tt / per_pass, r = tt % per_pass;
        const int shift = 8 * p;
        const uint64_t* kin = key_buf[(p + 1) & 1];
        const uint32_t* vin = val_buf[(p + 1) & 1];
        if (r < nh) {  // ---- histograms of blocks [r * kFbGroup, ...)
            if (p > 0) wait_at_least(&st->scatter_done[p - 1], nh, nullptr);
            const int b1 = (r + 1) * kFbGroup < nb ? (r + 1) * kFbGroup : nb;
            for (int b = r * kFbGroup; b < b1; b++) {
                for (int i = t; i < 256; i += kFbThreads) L.hist[i] = 0;
                __syncthreads();
                for (int i = t; i < kFbBlock; i += kFbThreads) {
                    const int64_t g = (int64_t)b * kFbBlock + i;
                    if (g < n) {
                        uint64_t k;
                        uint32_t v;
                        if (p == 0) {
                            job.load(g, k, v);
                            k -= kmin;
                        } else {
                            k = kin[g];
                        }
                        atomicAdd(&L.hist[(k >> shift) & 255u], 1u);
                    }
                }
                __syncthreads();
                for (int i = t; i < 256; i += kFbThreads) hist[(int64_t)i * nb + b] = L.hist[i];
            }
            signal_done(&st->hist_done[p]);
        } else if (r < nh + nseg) {  // ---- exclusive scan of one segment of the counters
            const int sg = r - nh;
            wait_at_least(&st->hist_done[p], nh, nullptr);
            const int64_t c0 = (int64_t)sg * kFbScanSeg;
            const int64_t len = n_counters - c0 < kFbScanSeg ? n_counters - c0 : kFbScanSeg;
            if (t == 0) L.misc = 0;
            __syncthreads();
            // segment total before the in-place exclusive scan overwrites it
            uint32_t part = 0;
            for (int64_t i = t; i < len; i += kFbThreads) part += hist[c0 + i];
            atomicAdd((uint32_t*)&L.misc, part);
            __syncthreads();
            radix_scan_counts(hist + c0, len, L);
            if (t == 0) seg_tot[sg] = (uint32_t)L.misc;
            signal_done(&st->seg_done[p]);
        } else if (r == nh + nseg) {  // ---- exclusive scan of the segment totals
            wait_at_least(&st->seg_done[p], nseg, nullptr);
            radix_scan_counts(seg_tot, nseg, L);
            signal_done(&st->scan_done[p]);
        } else {  // ---- stable scatter of blocks [h * kFbGroup, ...)
            const int h = r - nh - nseg - 1;
            wait_at_least(&st->scan_done[p], 1, nullptr);
            const int b1 = (h + 1) * kFbGroup < nb ? (h + 1) * kFbGroup : nb;
            for (int b = h * kFbGroup; b < b1; b++) {
            __syncthreads();  // the previous block's LDS is no longer read
            const int64_t g0 = (int64_t)b * kFbBlock;
            const int cntb = (int)((n - g0) < kFbBlock ? (n - g0) : kFbBlock);
            for (int i = t; i < kFbBlock; i += kFbThreads) {
                if (i < cntb) {
                    uint64_t k;
                    uint32_t v;
                    if (p == 0) {
                        job.load(g0 + i, k, v);
                        k -= kmin;
                    } else {
                        k = kin[g0 + i];
                        v = vin[g0 + i];
                    }
                    L.key[i] = k;
                    L.val[i] = v;
                    L.k0[i] = (uint32_t)((k >> shift) & 255u);
                } else {
                    L.k0[i] = 0xFFu;  // pads sort after every real element
                }
                L.v0[i] = (uint16_t)i;
            }
            for (int i = t; i < 256; i += kFbThreads) L.hist[i] = 0;
            __syncthreads();
            for (int i = t; i < cntb; i += kFbThreads) atomicAdd(&L.hist[L.k0[i]], 1u);
            __syncthreads();
            {
                const uint32_t c = t < 256 ? L.hist[t] : 0u;
                const uint32_t e = block_exclusive_scan<kFbThreads>(c, L.wsum, nullptr);
                if (t < 256) L.start[t] = e;
            }
            __syncthreads();
            const int which = block_radix_sort<kFbThreads, kFbBlock / kFbThreads>(L.k0, L.v0, L.k1, L.v1,
                                                                                  L.cnt, L.wsum, 8);
            const uint32_t* sk = which ? L.k1 : L.k0;
            const uint16_t* sv = which ? L.v1 : L.v0;
            const bool last = (p == passes - 1);
            uint64_t* kout = key_buf[p & 1];
            uint32_t* vout = val_buf[p & 1];
            for (int rr = t; rr < cntb; rr += kFbThreads) {
                const uint32_t d = sk[rr];
                const int e = sv[rr];
                const int64_t ci = (int64_t)d * nb + b;
                const int64_t pos = (int64_t)hist[ci] + seg_tot[ci / kFbScanSeg] + (rr - (int)L.start[d]);
                if (pos < 0 || pos >= n) {
                    atomicOr(err, 1);
                    continue;
                }
                if (last) job.store(pos, L.key[e], L.val[e]);
                if (!last || Job::kKeepSorted) {
                    kout[pos] = L.key[e];
                    vout[pos] = L.val[e];
                }
            }
            }  // blocks of the task
            signal_done(&st->scatter_done[p]);
        }
    }
}

}  // namespace hc
