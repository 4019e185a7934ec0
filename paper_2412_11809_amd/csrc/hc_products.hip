// Per-cluster products of a clustering, computed on the device from the
// outputs of hc_cluster (labels, feature table, cluster count):
//   * the bounding box of every cluster, the smallest sensor-aligned
//     rectangle holding its hits (the second, constant-time test of the
//     paper's merge cascade, Section 3.3);
//   * a filter over the feature rows (size, ToT sum, first ToA in closed
//     ranges), the data reduction of the paper's cluster-outputting stage
//     (Section 3.1; Section 6 names filtering among the tasks to move to the
//     GPU), as the ascending list of kept rows;
//   * the hits of the kept clusters grouped cluster by cluster, one block of
//     memory per cluster (what step 6 of the paper's high-level GPU algorithm
//     achieves by sorting clusters), blocks in ascending label order and the
//     hits of a block in input order.
// Kernels: row map + filter, box atomics, kept-row compaction with block
// starts, and a stable radix sort of the hits by kept rank (the ticketed
// engine of hc_radix.h).
#include <algorithm>

#include "hc_device.h"
#include "hc_radix.h"

namespace hc {

constexpr int kProdBlock = 2048;   // feature rows per compaction block
constexpr int kProdThreads = 256;

struct ProdStatus {
    int32_t err;       // a label or row out of range, or the cluster count is an error
    int32_t k;         // clusters (feature rows)
    int32_t n_keep;    // kept rows
    int32_t kept_hits; // hits of the kept clusters
    int32_t pad_[4];
    RadixState rs;
};

struct Prod {
    int32_t n;
    const hc_hit* hits;
    const int32_t* labels;
    const hc_features* feats;
    const int32_t* n_clusters;
    hc_filter filter;
    ProdStatus* st;
    int32_t* row_of;     // label -> feature row
    uint32_t* bx;        // per row: x_min, x_max, y_min, y_max
    uint8_t* keep;       // per row
    int32_t* kept_rank;  // per row: rank among the kept rows, -1 if dropped
    uint32_t* counts;    // per compaction block: kept rows, kept hits
    int32_t n_blocks;
    uint64_t* key[2];
    uint32_t* val[2];
    uint32_t* hist;
    int32_t nb;          // radix blocks
    // outputs (device; any may be null except keep_rows / n_keep)
    hc_box* boxes;
    int32_t* keep_rows;
    int32_t* n_keep;
    hc_hit* grouped;
    int32_t* grouped_idx;
    int64_t* row_start;
};

__global__ void k_prod_init(Prod a)
{
    int32_t* s = reinterpret_cast<int32_t*>(a.st);
    for (int i = threadIdx.x; i < (int)(sizeof(ProdStatus) / 4); i += blockDim.x) s[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t K = *a.n_clusters;
        if (K < 0 || K > a.n) {
            a.st->err = 1;
            a.st->k = 0;
        } else {
            a.st->k = K;
        }
    }
}

__device__ inline bool passes(const hc_filter& f, const hc_features& r)
{
    return r.size >= f.min_size && r.size <= f.max_size && r.sum_tot >= f.min_sum_tot &&
           r.sum_tot <= f.max_sum_tot && r.toa_min >= f.toa_from && r.toa_min <= f.toa_to;
}

// per feature row: where its label points, empty box, filter verdict
__global__ __launch_bounds__(256) void k_prod_rows(Prod a)
{
    const int K = a.st->k;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        const hc_features r = a.feats[k];
        if (r.label < 0 || r.label >= a.n) {
            atomicOr(&a.st->err, 1);
            a.keep[k] = 0;
            continue;
        }
        a.row_of[r.label] = k;
        a.bx[4 * (int64_t)k + 0] = 0xFFFFFFFFu;
        a.bx[4 * (int64_t)k + 1] = 0u;
        a.bx[4 * (int64_t)k + 2] = 0xFFFFFFFFu;
        a.bx[4 * (int64_t)k + 3] = 0u;
        a.keep[k] = passes(a.filter, r) ? 1 : 0;
    }
}

// Row of hit i's cluster (the feature row of its label), or -1.
__device__ inline int32_t prod_row(const Prod& a, int64_t i, int K)
{
    const int32_t lab = a.labels[i];
    if (lab < 0 || lab >= a.n) return -1;
    const int32_t r = a.row_of[lab];
    return (r >= 0 && r < K) ? r : -1;
}

// Boxes: the hits of one cluster are mostly consecutive in the input (it is
// nearly in ToA order), so each run of one row within a wave is reduced with
// shuffles first and only its last lane issues the four atomics.
__global__ __launch_bounds__(256) void k_prod_boxes(Prod a)
{
    const int K = a.st->k;
    if (a.st->err) return;
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < a.n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        int32_t r = -1;
        uint32_t x = 0, y = 0;
        if (i < a.n) {
            r = prod_row(a, i, K);
            if (r < 0) atomicOr(&a.st->err, 1);
            x = a.hits[i].x;
            y = a.hits[i].y;
        }
        uint32_t xmn = r >= 0 ? x : 0xFFFFFFFFu, xmx = x, ymn = r >= 0 ? y : 0xFFFFFFFFu, ymx = y;
        // suffix reductions over equal rows: after the loop the first lane of
        // each run (a lane whose left neighbour holds another row) has the run
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t ro = __shfl_down(r, o, kWave);
            const uint32_t a0 = __shfl_down(xmn, o, kWave), a1 = __shfl_down(xmx, o, kWave);
            const uint32_t a2 = __shfl_down(ymn, o, kWave), a3 = __shfl_down(ymx, o, kWave);
            // the lane o places to the right belongs to the same run only if
            // every row in between is equal; a run is contiguous, so comparing
            // the end points suffices
            if (lane + o < kWave && ro == r) {
                xmn = a0 < xmn ? a0 : xmn;
                xmx = a1 > xmx ? a1 : xmx;
                ymn = a2 < ymn ? a2 : ymn;
                ymx = a3 > ymx ? a3 : ymx;
            }
        }
        const int32_t rl = __shfl_up(r, 1, kWave);
        const bool head = lane == 0 || rl != r;
        if (head && r >= 0) {
            atomicMin(&a.bx[4 * (int64_t)r + 0], xmn);
            atomicMax(&a.bx[4 * (int64_t)r + 1], xmx);
            atomicMin(&a.bx[4 * (int64_t)r + 2], ymn);
            atomicMax(&a.bx[4 * (int64_t)r + 3], ymx);
        }
    }
}

__global__ __launch_bounds__(256) void k_prod_box_write(Prod a)
{
    const int K = a.st->k;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        hc_box b;
        b.x_min = (uint16_t)a.bx[4 * (int64_t)k + 0];
        b.x_max = (uint16_t)a.bx[4 * (int64_t)k + 1];
        b.y_min = (uint16_t)a.bx[4 * (int64_t)k + 2];
        b.y_max = (uint16_t)a.bx[4 * (int64_t)k + 3];
        a.boxes[k] = b;
    }
}

// kept rows and their hits per block of kProdBlock rows
__global__ __launch_bounds__(kProdThreads) void k_prod_count(Prod a)
{
    __shared__ uint32_t wsum[kProdThreads / kWave];
    const int K = a.st->k;
    const int64_t b0 = (int64_t)blockIdx.x * kProdBlock;
    if (b0 >= K) return;
    uint32_t c = 0, h = 0;
    for (int q = 0; q < kProdBlock / kProdThreads; q++) {
        const int64_t k = b0 + q * kProdThreads + threadIdx.x;
        if (k < K && a.keep[k]) {
            c++;
            h += a.feats[k].size;
        }
    }
    uint32_t tc, th;
    block_exclusive_scan<kProdThreads>(c, wsum, &tc);
    block_exclusive_scan<kProdThreads>(h, wsum, &th);
    if (threadIdx.x == 0) {
        a.counts[2 * blockIdx.x] = tc;
        a.counts[2 * blockIdx.x + 1] = th;
    }
}

__global__ __launch_bounds__(1024) void k_prod_scan(Prod a)
{
    __shared__ uint32_t wsum[1024 / kWave];
    const int K = a.st->k;
    const int nb = (K + kProdBlock - 1) / kProdBlock;
    uint32_t carry_c = 0, carry_h = 0;
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const uint32_t vc = i < nb ? a.counts[2 * i] : 0u;
        const uint32_t vh = i < nb ? a.counts[2 * i + 1] : 0u;
        uint32_t tc, th;
        const uint32_t ec = block_exclusive_scan<1024>(vc, wsum, &tc);
        const uint32_t eh = block_exclusive_scan<1024>(vh, wsum, &th);
        if (i < nb) {
            a.counts[2 * i] = carry_c + ec;
            a.counts[2 * i + 1] = carry_h + eh;
        }
        carry_c += tc;
        carry_h += th;
    }
    if (threadIdx.x == 0) {
        a.st->n_keep = (int32_t)carry_c;
        a.st->kept_hits = (int32_t)carry_h;
        if (a.n_keep) *a.n_keep = a.st->err ? HC_ERR_DEVICE : (int32_t)carry_c;
        if (a.row_start) a.row_start[carry_c] = carry_h;
    }
}

// kept rank of every row; kept rows in order; start of every kept block
__global__ __launch_bounds__(kProdThreads) void k_prod_scatter(Prod a)
{
    __shared__ uint32_t wsum[kProdThreads / kWave];
    constexpr int PER = kProdBlock / kProdThreads;
    const int K = a.st->k;
    const int64_t k0 = (int64_t)blockIdx.x * kProdBlock + (int64_t)threadIdx.x * PER;
    if ((int64_t)blockIdx.x * kProdBlock >= K) return;
    uint32_t c = 0, h = 0;
    for (int q = 0; q < PER; q++)
        if (k0 + q < K && a.keep[k0 + q]) {
            c++;
            h += a.feats[k0 + q].size;
        }
    uint32_t pc = a.counts[2 * blockIdx.x] + block_exclusive_scan<kProdThreads>(c, wsum, nullptr);
    uint32_t ph = a.counts[2 * blockIdx.x + 1] + block_exclusive_scan<kProdThreads>(h, wsum, nullptr);
    for (int q = 0; q < PER; q++) {
        const int64_t k = k0 + q;
        if (k >= K) break;
        if (a.keep[k]) {
            a.kept_rank[k] = (int32_t)pc;
            a.keep_rows[pc] = (int32_t)k;
            if (a.row_start) a.row_start[pc] = ph;
            pc++;
            ph += a.feats[k].size;
        } else {
            a.kept_rank[k] = -1;
        }
    }
}

// Stable sort of the hits by the kept rank of their cluster (dropped
// clusters sort behind every kept one); the sorted prefix of kept hits is
// written out.
struct GroupJob {
    static constexpr bool kKeepSorted = false;
    Prod a;
    __device__ int64_t count() const { return a.n; }
    __device__ void load(int64_t i, uint64_t& k, uint32_t& v) const
    {
        const int32_t r = prod_row(a, i, a.st->k);
        const int32_t kr = r >= 0 ? a.kept_rank[r] : -1;
        k = kr >= 0 ? (uint64_t)kr : (uint64_t)a.st->n_keep;
        v = (uint32_t)i;
    }
    __device__ int plan(RadixState& st, RadixLds&)
    {
        if (threadIdx.x == 0) {
            st.active = (a.st->err == 0 && a.st->n_keep > 0) ? 1 : 0;
            st.key_min = 0;
            const uint32_t top = (uint32_t)a.st->n_keep;
            const int bits = top == 0 ? 0 : 32 - __builtin_clz(top);
            st.passes = bits <= 8 ? 1 : (bits + 7) / 8;
        }
        return 0;
    }
    __device__ void store(int64_t pos, uint64_t, uint32_t v) const
    {
        if (pos < a.st->kept_hits) {
            if (a.grouped) a.grouped[pos] = a.hits[v];
            if (a.grouped_idx) a.grouped_idx[pos] = (int32_t)v;
        }
    }
    __device__ void extra(int, const uint64_t*, const uint32_t*, RadixLds&) {}
};

__global__ __launch_bounds__(kFbThreads) void k_prod_group(Prod a)
{
    if (a.st->err || a.st->n_keep == 0) return;
    GroupJob job{a};
    radix_engine(job, &a.st->rs, a.key, a.val, a.hist, a.nb, &a.st->err);
}

__global__ void k_prod_error(Prod a)
{
    if (threadIdx.x == 0 && a.st->err && a.n_keep) *a.n_keep = HC_ERR_DEVICE;
}

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// Workspace layout for n hits (pointers filled when base is non-null).
static size_t plan_products(int64_t n, Prod* a, char* base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += up256(bytes);
        return p;
    };
    const size_t N = (size_t)(n > 0 ? n : 1);
    a->n = (int32_t)n;
    a->st = (ProdStatus*)take(sizeof(ProdStatus));
    a->row_of = (int32_t*)take(4 * N);
    a->bx = (uint32_t*)take(16 * N);
    a->keep = (uint8_t*)take(N);
    a->kept_rank = (int32_t*)take(4 * N);
    a->n_blocks = (int32_t)((N + kProdBlock - 1) / kProdBlock);
    a->counts = (uint32_t*)take(8 * (size_t)a->n_blocks);
    a->nb = (int32_t)((N + kFbBlock - 1) / kFbBlock);
    a->key[0] = (uint64_t*)take(8 * N);
    a->key[1] = (uint64_t*)take(8 * N);
    a->val[0] = (uint32_t*)take(4 * N);
    a->val[1] = (uint32_t*)take(4 * N);
    a->hist = (uint32_t*)take(4 * (256 * (size_t)a->nb + fb_scan_segments(a->nb)));
    return off;
}

}  // namespace hc

using namespace hc;

extern "C" {

size_t hc_products_workspace_size(int64_t n)
{
    if (n < 0 || n > 0x7FFFFFFF) return 0;
    Prod a{};
    return plan_products(n, &a, nullptr);
}

int hc_cluster_products(const hc_hit* hits, int32_t n, const int32_t* labels, const hc_features* features,
                        const int32_t* n_clusters, const hc_filter* filter, hc_box* boxes, int32_t* keep_rows,
                        int32_t* n_keep, hc_hit* grouped, int32_t* grouped_idx, int64_t* row_start,
                        void* workspace, size_t workspace_bytes, void* stream)
{
    if (n < 0) return set_error(HC_ERR_ARG, "n < 0");
    if (!n_clusters || !keep_rows || !n_keep) return set_error(HC_ERR_ARG, "n_clusters, keep_rows and n_keep are required");
    if (n > 0 && (!hits || !labels || !features)) return set_error(HC_ERR_ARG, "hits, labels or features is NULL");
    Prod a{};
    const size_t need = plan_products(n, &a, nullptr);
    if (!workspace || workspace_bytes < need)
        return set_error(HC_ERR_WORKSPACE, "products workspace of " + std::to_string(workspace_bytes) +
                                               " bytes, need " + std::to_string(need));
    plan_products(n, &a, (char*)workspace);
    a.hits = hits;
    a.labels = labels;
    a.feats = features;
    a.n_clusters = n_clusters;
    if (filter) {
        a.filter = *filter;
    } else {
        a.filter.min_size = 0;
        a.filter.max_size = 0xFFFFFFFFu;
        a.filter.min_sum_tot = 0;
        a.filter.max_sum_tot = ~0ull;
        a.filter.toa_from = 0;
        a.filter.toa_to = ~0ull;
    }
    a.boxes = boxes;
    a.keep_rows = keep_rows;
    a.n_keep = n_keep;
    a.grouped = grouped;
    a.grouped_idx = grouped_idx;
    a.row_start = row_start;
    hipStream_t s = (hipStream_t)stream;
    const int g = n > 0 ? (int)std::min<int64_t>(((int64_t)n + 255) / 256, 4096) : 1;
    {
        TimedLaunch tl("products", s);
        hipLaunchKernelGGL(k_prod_init, dim3(1), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_prod_rows, dim3(g), dim3(256), 0, s, a);
        if (boxes) {
            hipLaunchKernelGGL(k_prod_boxes, dim3(g), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_prod_box_write, dim3(g), dim3(256), 0, s, a);
        }
        hipLaunchKernelGGL(k_prod_count, dim3(a.n_blocks), dim3(kProdThreads), 0, s, a);
        hipLaunchKernelGGL(k_prod_scan, dim3(1), dim3(1024), 0, s, a);
        hipLaunchKernelGGL(k_prod_scatter, dim3(a.n_blocks), dim3(kProdThreads), 0, s, a);
        if (grouped || grouped_idx)
            hipLaunchKernelGGL(k_prod_group, dim3(persistent_grid()), dim3(kFbThreads), 0, s, a);
        hipLaunchKernelGGL(k_prod_error, dim3(1), dim3(64), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HC_OK : set_device_error(e, "cluster products");
}

}  // extern "C"
