// Batch form: many independent chunks clustered by one launch sequence, an
// autotuner for its tiling choices, and HIP-graph capture of the sequence.
//
// Every kernel of the plain path maps its tile through the chunk table
// (tile_range), so one launch per stage covers all chunks with equally sized
// tiles whatever the chunk sizes: the chunk-to-work-group schedule is the
// tile table itself, balanced by construction.
#include <string.h>

#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hc_device.h"

namespace hc {

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// number of 32-bit words that differ between a and b
__global__ void k_count_diff(const uint32_t* a, const uint32_t* b, int64_t n, unsigned long long* out)
{
    unsigned long long c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += a[i] != b[i];
    if (c) atomicAdd(out, c);
}

}  // namespace hc

using namespace hc;

struct hc_batch_plan {
    uint32_t disorder_hint;
    int32_t xcd_map;
    int32_t link_mode;  // 0: default (pixel index when the bitmap fits), 1: pixel index, 2: window scan
    double time_ms;
};

struct hc_batch_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* ws = nullptr;
};

namespace {

// Pinned staging for the chunk/tile tables, reused once the previous upload
// has completed.
struct Staging {
    std::mutex mu;
    void* ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};
Staging g_stage;

int check_batch(const int64_t* offsets, int32_t n_chunks, const uint64_t* dts)
{
    if (n_chunks < 1 || !offsets || !dts) return set_error(HC_ERR_ARG, "batch needs n_chunks >= 1, offsets and dts");
    if (offsets[0] != 0) return set_error(HC_ERR_ARG, "offsets[0] must be 0");
    for (int c = 0; c < n_chunks; c++)
        if (offsets[c + 1] < offsets[c]) return set_error(HC_ERR_ARG, "offsets must not decrease");
    if (offsets[n_chunks] > 0x7FFFFFFF) return set_error(HC_ERR_OVERFLOW, "more than 2^31 - 1 hits in a batch");
    return HC_OK;
}

std::vector<SegSpec> make_segs(const int64_t* offsets, int32_t n_chunks, const uint64_t* dts)
{
    std::vector<SegSpec> v(n_chunks);
    for (int c = 0; c < n_chunks; c++)
        v[c] = SegSpec{offsets[c], (int32_t)(offsets[c + 1] - offsets[c]), dts[c], offsets[c]};
    return v;
}

uint32_t plan_hint(const hc_batch_plan* plan, const hc_opts* opts)
{
    if (plan) return plan->disorder_hint;
    return opts && opts->disorder_hint ? opts->disorder_hint : 4096;
}

int plan_batch(const int64_t* offsets, int32_t n_chunks, const uint64_t* dts, const hc_batch_plan* plan,
               const hc_opts* opts, std::vector<SegSpec>& segs, Work* w, char* base, size_t* bytes)
{
    const uint32_t W = opts && opts->width ? opts->width : 256;
    const uint32_t H = opts && opts->height ? opts->height : 256;
    if (W > 65535 || H > 65535 || (opts && !link_flags_valid(opts->flags)) || global_time_of(opts))
        return set_error(HC_ERR_ARG, "bad options (HC_FLAG_GLOBAL_TIME is for hc_cluster only)");
    segs = make_segs(offsets, n_chunks, dts);
    *bytes = plan_workspace(offsets[n_chunks], W, H, plan_hint(plan, opts), w, base, segs.data(), n_chunks);
    if (w) {
        w->xcd_map = plan ? plan->xcd_map : 1;
        w->link_mode = plan ? plan->link_mode : (link_mode_of(opts));
        if (n_chunks == 1) w->dt = dts[0];  // a one-chunk batch is the plain path
    }
    return HC_OK;
}

// Upload the chunk/tile tables through the pinned staging buffer.
int stage_tables(const Work& w, const std::vector<SegSpec>& segs, hipStream_t s)
{
    const size_t tb = segment_table_bytes(w);
    if (tb == 0) return HC_OK;
    std::lock_guard<std::mutex> lk(g_stage.mu);
    hipError_t e;
    if (g_stage.done && (e = hipEventSynchronize(g_stage.done)) != hipSuccess)
        return set_device_error(e, "staging event");
    if (g_stage.bytes < tb) {
        if (g_stage.ptr) (void)hipHostFree(g_stage.ptr);
        g_stage.ptr = nullptr;
        g_stage.bytes = 0;
        if ((e = hipHostMalloc(&g_stage.ptr, tb, hipHostMallocDefault)) != hipSuccess)
            return set_device_error(e, "hipHostMalloc(staging)");
        g_stage.bytes = tb;
    }
    if (!g_stage.done && (e = hipEventCreateWithFlags(&g_stage.done, hipEventDisableTiming)) != hipSuccess)
        return set_device_error(e, "hipEventCreate");
    int rc = upload_segments(w, segs.data(), (int)segs.size(), s, g_stage.ptr, g_stage.bytes);
    if (rc != HC_OK) return rc;
    if ((e = hipEventRecord(g_stage.done, s)) != hipSuccess) return set_device_error(e, "hipEventRecord");
    return HC_OK;
}

int enqueue_batch(const hc_hit* hits, int32_t n_chunks, int32_t* labels, hc_features* features,
                  int32_t* n_clusters, const Work& w, hipStream_t s)
{
    if (w.n == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, n_clusters, (int64_t)n_chunks, 0);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? HC_OK : set_device_error(e, "batch (empty)");
    }
    return enqueue_cluster(hits, w, labels, features, n_clusters, s);
}

}  // namespace

extern "C" {

size_t hc_batch_workspace_size(const int64_t* offsets, int32_t n_chunks, const hc_batch_plan* plan,
                               const hc_opts* opts)
{
    if (n_chunks < 1 || !offsets) return 0;
    std::vector<SegSpec> segs;
    std::vector<uint64_t> dts(n_chunks, 0);
    size_t bytes = 0;
    if (plan_batch(offsets, n_chunks, dts.data(), plan, opts, segs, nullptr, nullptr, &bytes) != HC_OK) return 0;
    return bytes;
}

int hc_cluster_batch(const hc_hit* hits, const int64_t* offsets, int32_t n_chunks, const uint64_t* dts,
                     int32_t* labels, hc_features* features, int32_t* n_clusters, const hc_batch_plan* plan,
                     const hc_opts* opts)
{
    int rc = check_batch(offsets, n_chunks, dts);
    if (rc != HC_OK) return rc;
    const int64_t n = offsets[n_chunks];
    if (!n_clusters || (n > 0 && (!hits || !labels))) return set_error(HC_ERR_ARG, "NULL buffer");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    std::vector<SegSpec> segs;
    Work w;
    size_t need = 0;
    if ((rc = plan_batch(offsets, n_chunks, dts, plan, opts, segs, &w, nullptr, &need)) != HC_OK) return rc;
    void* ws = opts ? opts->workspace : nullptr;
    std::unique_lock<std::mutex> hold;  // a cached workspace stays ours until the launches are enqueued
    if (ws) {
        if (opts->workspace_bytes < need) return set_error(HC_ERR_WORKSPACE, "batch workspace too small");
    } else if ((rc = cached_workspace(need, s, &ws, &hold)) != HC_OK) {
        return rc;
    }
    if ((rc = plan_batch(offsets, n_chunks, dts, plan, opts, segs, &w, (char*)ws, &need)) != HC_OK) return rc;
    if ((rc = stage_tables(w, segs, s)) != HC_OK) return rc;
    return enqueue_batch(hits, n_chunks, labels, features, n_clusters, w, s);
}

int hc_batch_plan_describe(const hc_batch_plan* plan, char* buf, size_t cap)
{
    if (!plan || !buf || cap == 0) return set_error(HC_ERR_ARG, "NULL plan or buffer");
    const int T = sort_tile_for(plan->disorder_hint ? plan->disorder_hint : 4096);
    snprintf(buf, cap, "disorder_hint=%u sort_tile=%d xcd_map=%d link=%s time_ms=%.4f", plan->disorder_hint, T,
             plan->xcd_map, plan->link_mode == 1 ? "index" : plan->link_mode == 2 ? "window" : "default",
             plan->time_ms);
    return HC_OK;
}

void hc_batch_plan_destroy(hc_batch_plan* plan) { delete plan; }

int hc_batch_autotune(const hc_hit* hits, const int64_t* offsets, int32_t n_chunks, const uint64_t* dts,
                      int32_t* labels, hc_features* features, int32_t* n_clusters, const hc_opts* opts,
                      hc_batch_plan** out)
{
    if (!out) return set_error(HC_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_batch(offsets, n_chunks, dts);
    if (rc != HC_OK) return rc;
    const int64_t n = offsets[n_chunks];
    if (!n_clusters || !labels || !features || n == 0) return set_error(HC_ERR_ARG, "autotune needs outputs and hits");
    static std::mutex cache_mu;
    static std::map<std::tuple<int, int, int>, hc_batch_plan> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    int lg = 0;
    while ((1ll << (lg + 1)) <= n) lg++;
    const auto key = std::make_tuple(dev, lg, n_chunks);
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *out = new hc_batch_plan(it->second);
            return hc_cluster_batch(hits, offsets, n_chunks, dts, labels, features, n_clusters, *out, opts);
        }
    }
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    hipError_t e;
    // reference outputs of the default plan
    int32_t *ref_lab = nullptr, *ref_cnt = nullptr;
    hc_features* ref_feat = nullptr;
    unsigned long long* diff = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(ref_lab);
        (void)hipFree(ref_cnt);
        (void)hipFree(ref_feat);
        (void)hipFree(diff);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if ((e = hipMalloc(&ref_lab, 4 * n)) != hipSuccess || (e = hipMalloc(&ref_cnt, 4 * (size_t)n_chunks)) != hipSuccess ||
        (e = hipMalloc(&ref_feat, sizeof(hc_features) * n)) != hipSuccess ||
        (e = hipMalloc(&diff, sizeof(unsigned long long))) != hipSuccess || (e = hipEventCreate(&e0)) != hipSuccess ||
        (e = hipEventCreate(&e1)) != hipSuccess) {
        cleanup();
        return set_device_error(e, "autotune allocation");
    }
    const int64_t fw = (int64_t)n * (sizeof(hc_features) / 4);
    auto run = [&](const hc_batch_plan* p) -> int {
        hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, (uint32_t*)features, fw, 0u);
        return hc_cluster_batch(hits, offsets, n_chunks, dts, labels, features, n_clusters, p, opts);
    };
    hc_batch_plan base{plan_hint(nullptr, opts), 1, 0, 0.0};
    if ((rc = run(&base)) != HC_OK) {
        cleanup();
        return rc;
    }
    (void)hipMemcpyAsync(ref_lab, labels, 4 * n, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(ref_cnt, n_clusters, 4 * (size_t)n_chunks, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(ref_feat, features, sizeof(hc_features) * n, hipMemcpyDeviceToDevice, s);
    const uint32_t hints[] = {512, 1024, 2048, 4096, 8192, 16384};
    hc_batch_plan best{0, 0, 0, 1e30};
    for (uint32_t h : hints) {
        for (int cfg = 0; cfg < 4; cfg++) {  // link mode: default, window scan
            hc_batch_plan cand{h, 1 - (cfg & 1), (cfg >> 1) ? 2 : 0, 0.0};
            if ((rc = run(&cand)) != HC_OK) break;  // warm-up (and the parity check below)
            unsigned long long nd = 0;
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)diff, (int64_t)2, 0u);
            hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, s, (const uint32_t*)labels, (const uint32_t*)ref_lab,
                               n, diff);
            hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, s, (const uint32_t*)features,
                               (const uint32_t*)ref_feat, fw, diff);
            hipLaunchKernelGGL(k_count_diff, dim3(1), dim3(256), 0, s, (const uint32_t*)n_clusters,
                               (const uint32_t*)ref_cnt, (int64_t)n_chunks, diff);
            (void)hipMemcpyAsync(&nd, diff, sizeof(nd), hipMemcpyDeviceToHost, s);
            if ((e = hipStreamSynchronize(s)) != hipSuccess) {
                rc = set_device_error(e, "autotune");
                break;
            }
            if (nd != 0) continue;  // a candidate that changes any output bit is never chosen
            const int reps = 3;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && rc == HC_OK; r++)
                rc = hc_cluster_batch(hits, offsets, n_chunks, dts, labels, features, n_clusters, &cand, opts);
            (void)hipEventRecord(e1, s);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                rc = set_device_error(e, "autotune timing");
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            cand.time_ms = ms / reps;
            if (cand.time_ms < best.time_ms) best = cand;
        }
        if (rc != HC_OK) break;
    }
    cleanup();
    if (rc != HC_OK) return rc;
    if (best.time_ms >= 1e29) return set_error(HC_ERR_DEVICE, "autotune: no candidate reproduced the reference");
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        cache[key] = best;
    }
    *out = new hc_batch_plan(best);
    // leave the chosen plan's result in the outputs
    return hc_cluster_batch(hits, offsets, n_chunks, dts, labels, features, n_clusters, *out, opts);
}

int hc_batch_graph_create(const hc_hit* hits, const int64_t* offsets, int32_t n_chunks, const uint64_t* dts,
                          int32_t* labels, hc_features* features, int32_t* n_clusters,
                          const hc_batch_plan* plan, const hc_opts* opts, hc_batch_graph** out)
{
    if (!out) return set_error(HC_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_batch(offsets, n_chunks, dts);
    if (rc != HC_OK) return rc;
    const int64_t n = offsets[n_chunks];
    if (!n_clusters || (n > 0 && (!hits || !labels))) return set_error(HC_ERR_ARG, "NULL buffer");
    std::vector<SegSpec> segs;
    Work w;
    size_t need = 0;
    if ((rc = plan_batch(offsets, n_chunks, dts, plan, opts, segs, &w, nullptr, &need)) != HC_OK) return rc;
    hc_batch_graph* g = new hc_batch_graph();
    hipError_t e;
    hipStream_t cs = nullptr;
    auto fail_out = [&](int code) {
        if (cs) (void)hipStreamDestroy(cs);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        (void)hipFree(g->ws);
        delete g;
        return code;
    };
    if ((e = hipMalloc(&g->ws, need)) != hipSuccess) return fail_out(set_device_error(e, "hipMalloc(graph workspace)"));
    if ((rc = plan_batch(offsets, n_chunks, dts, plan, opts, segs, &w, (char*)g->ws, &need)) != HC_OK)
        return fail_out(rc);
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
        return fail_out(set_device_error(e, "hipStreamCreate"));
    // the tables are constant: upload them once, outside the graph
    if ((rc = stage_tables(w, segs, cs)) != HC_OK) return fail_out(rc);
    if ((e = hipStreamSynchronize(cs)) != hipSuccess) return fail_out(set_device_error(e, "hipStreamSynchronize"));
    const bool timing = timing_set(false);  // no event records inside the graph
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        timing_set(timing);
        return fail_out(set_device_error(e, "hipStreamBeginCapture"));
    }
    rc = enqueue_batch(hits, n_chunks, labels, features, n_clusters, w, cs);
    e = hipStreamEndCapture(cs, &g->graph);
    timing_set(timing);
    if (rc != HC_OK) return fail_out(rc);
    if (e != hipSuccess) return fail_out(set_device_error(e, "hipStreamEndCapture"));
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
        return fail_out(set_device_error(e, "hipGraphInstantiate"));
    (void)hipStreamDestroy(cs);
    *out = g;
    return HC_OK;
}

int hc_batch_graph_launch(hc_batch_graph* g, void* stream)
{
    if (!g || !g->exec) return set_error(HC_ERR_ARG, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    return e == hipSuccess ? HC_OK : set_device_error(e, "hipGraphLaunch");
}

void hc_batch_graph_destroy(hc_batch_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipFree(g->ws);
    delete g;
}

}  // extern "C"
