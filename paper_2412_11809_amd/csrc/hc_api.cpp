// C-ABI of the hit-clustering library: argument checking, workspace layout,
// the launch sequence of hc_cluster, error strings and kernel timing.
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hc.h"
#include "hc_internal.h"

namespace hc {

static thread_local std::string g_err;

static int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

static int device_fail(hipError_t e, const char* what)
{
    return fail(HC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------ workspace
static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int64_t tiles_of(int64_t count, int size) { return (count + size - 1) / size; }

size_t plan_workspace(int64_t n, uint32_t width, uint32_t height, uint32_t disorder, Work* w, char* base,
                      const SegSpec* segs, int n_seg)
{
    Work x{};
    x.n = (int32_t)n;
    x.width = width;
    x.height = height;
    x.n_seg = n_seg < 1 ? 1 : n_seg;
    x.xcd_map = 1;
    x.link_mode = 0;
    const int64_t D = disorder ? disorder : 4096;
    const int T = sort_tile_for(D);
    x.sort_tile = T;
    x.sort_ipt = T / kSortThreads;
    int64_t m = (2 * D + T - 1) / T;
    if (m < 1) m = 1;
    x.force_fallback = m > kMaxNeighbourTiles ? 1 : 0;
    x.sort_m = (int32_t)(m > kMaxNeighbourTiles ? kMaxNeighbourTiles : m);
    const int sizes[4] = {T, kLinkTile, kFeatTile, kScanBlock};
    int64_t nt[4] = {0, 0, 0, 0};
    if (x.n_seg == 1) {
        for (int k = 0; k < 4; k++) nt[k] = tiles_of(n, sizes[k]);
    } else {
        for (int sg = 0; sg < n_seg; sg++)
            for (int k = 0; k < 4; k++) nt[k] += tiles_of(segs[sg].count, sizes[k]);
    }
    x.n_sort_tiles = (int32_t)nt[0];
    x.n_link_tiles = (int32_t)nt[1];
    x.n_feat_tiles = (int32_t)nt[2];
    x.n_scan_blocks = (int32_t)nt[3];
    x.n_fb_blocks = (int32_t)((n + kFbBlock - 1) / kFbBlock);
    x.edge_cap = (int64_t)x.n_link_tiles * kLinkHaloCap;
    x.carry_cap = (int64_t)x.n_feat_tiles * kFeatHash;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return base ? base + at : nullptr;
    };
    const size_t N = (size_t)n;
    x.status = (Status*)take(sizeof(Status));
    if (x.n_seg > 1) {
        // one contiguous region: chunk table, then the chunk of every tile per kind
        size_t tb = align_up(sizeof(SegInfo) * (size_t)x.n_seg, 16);
        for (int k = 0; k < 4; k++) tb += align_up(4 * (size_t)nt[k], 16);
        char* r = (char*)take(tb);
        x.segs = (SegInfo*)r;
        size_t at = align_up(sizeof(SegInfo) * (size_t)x.n_seg, 16);
        for (int k = 0; k < 4; k++) {
            x.tile_seg[k] = r ? (int32_t*)(r + at) : nullptr;
            at += align_up(4 * (size_t)nt[k], 16);
        }
    }
    x.tiles = (TileInfo*)take(sizeof(TileInfo) * (size_t)x.n_sort_tiles);
    x.tile_q = (uint32_t*)take(4 * (size_t)kTileQ * (size_t)x.n_sort_tiles);
    x.ts_rel = (uint32_t*)take(4 * N);
    x.ts_pay = (uint2*)take(8 * N);
    x.s_toa = (uint64_t*)take(8 * N);
    x.s_xy = (uint32_t*)take(4 * N);
    x.s_tot = (uint16_t*)take(2 * N);
    x.s_idx = (int32_t*)take(4 * N);
    x.link_h0 = (int32_t*)take(4 * (size_t)x.n_link_tiles);
    x.gparent = (int32_t*)take(4 * N);
    x.edges = (int2*)take(sizeof(int2) * (size_t)x.edge_cap);
    x.tile_nedge = (int32_t*)take(4 * (size_t)x.n_link_tiles);
    x.overflow_tiles = (int32_t*)take(4 * (size_t)x.n_link_tiles);
    x.deep_tiles = (int32_t*)take(4 * (size_t)x.n_link_tiles);
    x.deep_ws = (int32_t*)take(4 * (size_t)x.n_link_tiles);
    x.run_off = (int32_t*)take(4 * ((size_t)x.n_link_tiles + 1));
    x.run_base = (int32_t*)take(4 * (size_t)x.n_link_tiles);
    x.blk_run = (int32_t*)take(4 * ((size_t)x.n_fb_blocks + 1));
    x.slots = (SlotRec*)take(sizeof(SlotRec) * N);
    x.carries = (SlotRec*)take(sizeof(SlotRec) * (size_t)x.carry_cap);
    x.tile_ncarry = (int32_t*)take(4 * (size_t)x.n_feat_tiles);
    x.blk_count = (uint32_t*)take(4 * (size_t)x.n_scan_blocks);
    x.blk_off = (uint32_t*)take(4 * (size_t)x.n_scan_blocks + 4);
    x.root_mask = (unsigned long long*)take(8 * (size_t)x.n_scan_blocks * (kScanBlock / 64));
    x.root_wpre = (uint16_t*)take(2 * (size_t)x.n_scan_blocks * (kScanBlock / 64));
    x.fb_key[0] = (uint64_t*)take(8 * N);
    x.fb_key[1] = (uint64_t*)take(8 * N);
    x.fb_val[0] = (uint32_t*)take(4 * N);
    x.fb_val[1] = (uint32_t*)take(4 * N);
    // digit counters, then one total per scan segment
    x.fb_hist = (uint32_t*)take(4 * (256 * (size_t)x.n_fb_blocks + fb_scan_segments(x.n_fb_blocks)));
    if (w) *w = x;
    return off;
}

size_t segment_table_bytes(const Work& w)
{
    if (w.n_seg <= 1) return 0;
    const int64_t nt[4] = {w.n_sort_tiles, w.n_link_tiles, w.n_feat_tiles, w.n_scan_blocks};
    size_t tb = align_up(sizeof(SegInfo) * (size_t)w.n_seg, 16);
    for (int k = 0; k < 4; k++) tb += align_up(4 * (size_t)nt[k], 16);
    return tb;
}

int upload_segments(const Work& w, const SegSpec* segs, int n_seg, hipStream_t s, void* staging,
                    size_t staging_bytes)
{
    if (w.n_seg <= 1) return HC_OK;
    const size_t tb = segment_table_bytes(w);
    if (!staging || staging_bytes < tb) return fail(HC_ERR_ARG, "segment staging buffer too small");
    char* h = (char*)staging;
    SegInfo* si = (SegInfo*)h;
    const int sizes[4] = {w.sort_tile, kLinkTile, kFeatTile, kScanBlock};
    int32_t* ts[4];
    size_t at = align_up(sizeof(SegInfo) * (size_t)n_seg, 16);
    const int64_t nt[4] = {w.n_sort_tiles, w.n_link_tiles, w.n_feat_tiles, w.n_scan_blocks};
    for (int k = 0; k < 4; k++) {
        ts[k] = (int32_t*)(h + at);
        at += align_up(4 * (size_t)nt[k], 16);
    }
    int64_t t0[4] = {0, 0, 0, 0};
    for (int sg = 0; sg < n_seg; sg++) {
        SegInfo& r = si[sg];
        r.start = segs[sg].start;
        r.count = segs[sg].count;
        r.pad_ = 0;
        r.dt = segs[sg].dt;
        r.out = segs[sg].out;
        r.toa_min = ~0ull;
        for (int k = 0; k < 4; k++) {
            r.tile0[k] = (int32_t)t0[k];
            const int64_t c = tiles_of(segs[sg].count, sizes[k]);
            for (int64_t q = 0; q < c; q++) ts[k][t0[k] + q] = sg;
            t0[k] += c;
        }
    }
    hipError_t e = hipMemcpyAsync(w.segs, h, tb, hipMemcpyHostToDevice, s);
    return e == hipSuccess ? HC_OK : device_fail(e, "segment table upload");
}

// One cached workspace per (device, stream) for callers that pass none.
// Work on one stream runs in order, so calls on that stream may share its
// buffer; calls on different streams never share one.  The entry's lock is
// held by the caller until its launches are enqueued, so a call that grows
// the buffer (after synchronising the stream: every earlier user enqueued its
// work there before releasing the lock) never frees memory that another
// thread is about to hand to a kernel.
struct CachedWs {
    std::mutex mu;
    void* ptr = nullptr;
    size_t bytes = 0;
};
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, std::unique_ptr<CachedWs>> g_ws;

int cached_workspace(size_t need, hipStream_t s, void** out, std::unique_lock<std::mutex>* hold)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    CachedWs* c;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        std::unique_ptr<CachedWs>& slot = g_ws[std::make_pair(dev, s)];
        if (!slot) slot.reset(new CachedWs());
        c = slot.get();
    }
    std::unique_lock<std::mutex> lk(c->mu);
    if (c->bytes < need) {
        if (c->ptr) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return device_fail(e, "hipStreamSynchronize");
            (void)hipFree(c->ptr);
            c->ptr = nullptr;
            c->bytes = 0;
        }
        e = hipMalloc(&c->ptr, need);
        if (e != hipSuccess) return device_fail(e, "hipMalloc(workspace)");
        c->bytes = need;
    }
    *out = c->ptr;
    *hold = std::move(lk);
    return HC_OK;
}

int persistent_grid()
{
    static std::mutex mu;
    static std::vector<int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cus.size() <= dev) cus.resize(dev + 1, 0);
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// ---------------------------------------------------------------- timing
struct TimingRec {
    const char* name;
    hipEvent_t start, stop;
};
static bool g_timing = false;
static std::string g_tsel;  // time only launches of this kernel name (empty: all)
static std::mutex g_tmu;  // launches from several host threads (server workers)
static std::vector<TimingRec> g_trecs;
static size_t g_tused = 0;

bool timing_set(bool on)
{
    const bool prev = g_timing;
    g_timing = on;
    return prev;
}

TimedLaunch::TimedLaunch(const char* name, hipStream_t s) : name_(name), s_(s), slot_(-1)
{
    if (!g_timing) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_tsel.empty() && g_tsel != name) return;
    if (g_tused == g_trecs.size()) {
        TimingRec r{name, nullptr, nullptr};
        if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return;
        g_trecs.push_back(r);
    }
    slot_ = (int)g_tused++;
    g_trecs[slot_].name = name;
    (void)hipEventRecord(g_trecs[slot_].start, s);
}

TimedLaunch::~TimedLaunch()
{
    if (slot_ < 0) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    (void)hipEventRecord(g_trecs[slot_].stop, s_);
}

int set_error(int code, const std::string& msg) { return fail(code, msg); }
int set_device_error(hipError_t e, const char* what) { return device_fail(e, what); }

int enqueue_cluster(const hc_hit* hits, const Work& w, int32_t* labels, hc_features* features,
                    int32_t* n_clusters, hipStream_t s)
{
    hipError_t e;
#define HC_LAUNCH(call, what)                                        \
    do {                                                             \
        if ((e = (call)) != hipSuccess) return device_fail(e, what); \
    } while (0)
    HC_LAUNCH(launch_init(w, s), "init");
    HC_LAUNCH(launch_tile_sort(hits, w, s), "tile_sort");
    if (!w.force_fallback) HC_LAUNCH(launch_tile_merge(w, s), "tile_merge");
    HC_LAUNCH(launch_sort_fallback(hits, w, s), "sort_fallback");
    HC_LAUNCH(launch_link_halo(w, s), "link_halo");
    HC_LAUNCH(launch_link(w, s), "link");
    HC_LAUNCH(launch_link_wide(w, s), "link_wide");
    HC_LAUNCH(launch_link_fallback(w, s), "link_fallback");
    HC_LAUNCH(launch_union_edges(w, s), "union_edges");
    HC_LAUNCH(launch_flatten(w, labels, s), "flatten");
    HC_LAUNCH(launch_scan_blocks(w, n_clusters, s), "scan_blocks");  // cluster ranks, before the records
    if (features) {
        HC_LAUNCH(launch_features(w, labels, s), "features");
        HC_LAUNCH(launch_carries(w, s), "carries");
        HC_LAUNCH(launch_compact(w, features, s), "compact");
    }
#undef HC_LAUNCH
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" {

const char* hc_last_error(void) { return g_err.c_str(); }

const char* hc_version(void) { return "hc 0.1 (gfx950)"; }

size_t hc_workspace_size(const hc_opts* opts, int64_t n)
{
    if (n < 0) return 0;
    const uint32_t W = opts && opts->width ? opts->width : 256;
    const uint32_t H = opts && opts->height ? opts->height : 256;
    const size_t base = plan_workspace(n, W, H, opts ? opts->disorder_hint : 0, nullptr, nullptr);
    return global_time_of(opts) ? base + plan_global(n, nullptr, nullptr) : base;
}

int hc_cluster(const hc_hit* hits, int32_t n, uint64_t dt, int32_t* labels, hc_features* features,
               int32_t* n_clusters, const hc_opts* opts)
{
    if (n < 0) return fail(HC_ERR_ARG, "n < 0");
    if (!n_clusters) return fail(HC_ERR_ARG, "n_clusters is NULL");
    if (n > 0 && (!hits || !labels)) return fail(HC_ERR_ARG, "hits or labels is NULL");
    const uint32_t W = opts && opts->width ? opts->width : 256;
    const uint32_t H = opts && opts->height ? opts->height : 256;
    if (W > 65535 || H > 65535) return fail(HC_ERR_ARG, "sensor dimensions must be 1..65535");
    if (opts && !link_flags_valid(opts->flags)) return fail(HC_ERR_ARG, "unknown flags");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    hipError_t e;
    if (n == 0) {
        if ((e = launch_write_count(n_clusters, 0, s)) != hipSuccess) return device_fail(e, "write_count");
        return HC_OK;
    }
    Work w;
    const uint32_t D = opts ? opts->disorder_hint : 0;
    const bool global = global_time_of(opts);
    const size_t base_need = plan_workspace(n, W, H, D, &w, nullptr);
    const size_t need = global ? base_need + plan_global(n, nullptr, nullptr) : base_need;
    void* ws = opts ? opts->workspace : nullptr;
    std::unique_lock<std::mutex> hold;  // a cached workspace stays ours until the launches are enqueued
    if (ws) {
        if (opts->workspace_bytes < need)
            return fail(HC_ERR_WORKSPACE, "workspace of " + std::to_string(opts->workspace_bytes) +
                                              " bytes, need " + std::to_string(need));
    } else {
        int rc = cached_workspace(need, s, &ws, &hold);
        if (rc != HC_OK) return rc;
    }
    plan_workspace(n, W, H, D, &w, (char*)ws);
    w.dt = dt;
    w.link_mode = link_mode_of(opts);
    if (global) return global_cluster(hits, w, (char*)ws + base_need, labels, features, n_clusters, s);
    return enqueue_cluster(hits, w, labels, features, n_clusters, s);
}

int hc_timing_enable(int on)
{
    g_timing = on != 0;
    return HC_OK;
}

int hc_timing_select(const char* name)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_tsel = name ? name : "";
    return HC_OK;
}

int hc_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_tused = 0;
    return HC_OK;
}

int hc_timing_read(const char** names, int64_t* launches, double* total_ms, int32_t cap)
{
    std::vector<const char*> nm;
    std::vector<int64_t> cnt;
    std::vector<double> ms;
    std::lock_guard<std::mutex> lk(g_tmu);
    for (size_t i = 0; i < g_tused; i++) {
        TimingRec& r = g_trecs[i];
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return device_fail(e, "hipEventSynchronize");
        float t = 0.f;
        e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) return device_fail(e, "hipEventElapsedTime");
        size_t k = 0;
        while (k < nm.size() && std::string(nm[k]) != r.name) k++;
        if (k == nm.size()) {
            nm.push_back(r.name);
            cnt.push_back(0);
            ms.push_back(0.0);
        }
        cnt[k]++;
        ms[k] += t;
    }
    for (size_t k = 0; k < nm.size() && (int32_t)k < cap; k++) {
        if (names) names[k] = nm[k];
        if (launches) launches[k] = cnt[k];
        if (total_ms) total_ms[k] = ms[k];
    }
    return (int)nm.size();
}

}  // extern "C"
