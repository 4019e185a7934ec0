// Host ingest front end: the paper's hit buffer filling (its Algorithm
// "Hit buffer filling", Section 4.1) feeding the stream form through pinned,
// multi-buffered copies that overlap with the clustering (steps 1, 2 and 8 of
// its high-level GPU algorithm; pinned memory and copy/compute overlap are
// the optimisations it lists in Section 5).
//
// Hits arrive in detector order (t-ordered, Section 3.1) and are numbered by
// arrival.  A buffer first takes hits freely up to b - b_t of them, tracking
// the largest ToA seen (toa_max); after that it takes only hits with
// toa < toa_max + t_closing, and later hits go to the next buffer; once a hit
// arrives with toa - toa_max > t + t_closing no later hit can belong to the
// buffer any more, and it is sent.  Each sent buffer is copied to the device
// on a copy stream and pushed into an hc_stream with the hits' arrival
// indices as ids, so every label is the smallest arrival index of its
// cluster whatever buffer a hit travelled in; clusters that span buffers are
// stitched by the stream.  When a buffer's chunk is complete, its labels are
// copied back and placed at their arrival indices in the caller's array.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <string.h>

#include <atomic>
#include <deque>
#include <string>
#include <vector>

#include "hc.h"
#include "hc_internal.h"

using namespace hc;

namespace {

// One buffer: pinned host hits and runs of arrival indices, their device copies,
// from filling until the push that reads them has run on the device.
struct Slot {
    hc_hit* h_hits = nullptr;
    int2* h_runs = nullptr;       // arrival ids as runs: (position, id) where a run starts
    int32_t n_runs = 0;
    hc_hit* d_hits = nullptr;
    int32_t* d_ids = nullptr;
    int2* d_runs = nullptr;
    hipEvent_t copied = nullptr;  // the H2D copy has read the host buffer
    int64_t count = 0;
    uint64_t push = 0;            // stream push that reads the device copies
    enum { kFree, kFilling, kPushed } state = kFree;
};

// One sent buffer until its labels are all final: where the device writes
// them, the arrival ids as runs (position, id) of consecutive ids, and its
// number of hits.
struct Chunk {
    uint64_t seq = 0;
    int32_t* d_labels = nullptr;
    std::vector<int2> runs;
    int64_t count = 0;
};

// Per-hit arrival ids of a buffer from its runs: position i takes the id of
// the last run starting at or before it, plus its distance from that start.
__global__ void k_ingest_ids(const int2* __restrict__ runs, int32_t n_runs, int32_t count, int32_t* ids)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || n_runs <= 0) return;
    int32_t lo = 0, hi = n_runs;  // the first run starting after i
    while (lo < hi) {
        const int32_t m = (lo + hi) >> 1;
        if (runs[m].x <= i) lo = m + 1; else hi = m;
    }
    const int2 r = runs[lo > 0 ? lo - 1 : 0];
    ids[i] = r.y + (i - r.x);
}

}  // namespace

struct hc_ingest {
    hc_ingest_config cfg{};
    hc_stream* st = nullptr;
    hipStream_t s = nullptr;   // pushes
    hipStream_t cs = nullptr;  // host-to-device copies
    hipStream_t ls = nullptr;  // labels back to the host
    std::vector<Slot> slots;
    std::deque<Chunk> chunks;          // sent, labels not yet all final
    std::vector<int32_t*> label_pool;  // device label buffers of b entries, free
    int32_t* h_labels = nullptr;       // pinned staging of one buffer's labels
    int cur = -1, nxt = -1;    // the buffer being filled and the next buffer
    uint64_t toa_max = 0;
    bool has_max = false;
    int64_t fed = 0;           // hits numbered so far
    uint64_t seq = 0;          // buffers sent
    int32_t* labels_out = nullptr;
    int64_t labels_cap = 0;
    hc_ingest_stats stats{};
    bool failed = false;
    std::vector<uint64_t> tags;
    std::vector<int32_t> status;
};

static int fail_ing(hc_ingest* g, int code, const std::string& msg)
{
    g->failed = true;
    return set_error(code, msg);
}

// Copy m hits into a buffer and return the largest ToA among them and mx.
// Streaming stores: a buffer of several MiB does not stay in the CPU caches
// until the device reads it, and ordinary stores would first read every
// line they write (about three times slower for 2M-hit buffers).
static uint64_t copy_hits_max(hc_hit* dst, const hc_hit* src, int64_t m, uint64_t mx)
{
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    static_assert(sizeof(hc_hit) == sizeof(u64x2) && offsetof(hc_hit, toa) == 0, "a hit is two words, ToA first");
    for (int64_t j = 0; j < m; j++) {
        u64x2 v;
        ::memcpy(&v, src + j, sizeof(v));
        __builtin_nontemporal_store(v, reinterpret_cast<u64x2*>(dst + j));
        mx = v.x > mx ? v.x : mx;
    }
    std::atomic_thread_fence(std::memory_order_seq_cst);  // the streaming stores complete before the copy is sent
    return mx;
}

static void free_slot(Slot& sl)
{
    if (sl.h_hits) (void)hipHostFree(sl.h_hits);
    if (sl.h_runs) (void)hipHostFree(sl.h_runs);
    (void)hipFree(sl.d_hits);
    (void)hipFree(sl.d_ids);
    (void)hipFree(sl.d_runs);
    if (sl.copied) (void)hipEventDestroy(sl.copied);
}

// Labels of the completed buffers back to the host, placed by arrival index;
// buffers whose push has run are free again.
static int collect(hc_ingest* g)
{
    const uint64_t ran = stream_pushes_retired(g->st);
    for (Slot& sl : g->slots)
        if (sl.state == Slot::kPushed && sl.push < ran) sl.state = Slot::kFree;
    int32_t nd = 0;
    const int cap = (int)g->tags.size();
    for (;;) {
        if (hc_stream_poll(g->st, g->tags.data(), g->status.data(), cap, &nd, nullptr, 0, nullptr) != HC_OK)
            return fail_ing(g, HC_ERR_DEVICE, std::string("ingest: ") + hc_last_error());
        for (int32_t k = 0; k < nd; k++) {
            auto it = g->chunks.begin();
            while (it != g->chunks.end() && it->seq != g->tags[k]) ++it;
            if (it == g->chunks.end()) continue;
            if (g->status[k] != HC_OK)
                return fail_ing(g, g->status[k], "ingest: a buffer was rejected (input not t-ordered within t?)");
            const int64_t m = it->count;
            hipError_t e = hipMemcpyAsync(g->h_labels, it->d_labels, 4 * (size_t)m, hipMemcpyDeviceToHost, g->ls);
            if (e == hipSuccess) e = hipStreamSynchronize(g->ls);
            if (e != hipSuccess) return fail_ing(g, HC_ERR_DEVICE, "ingest: label copy");
            // place by arrival index, one copy per run of consecutive indices
            const std::vector<int2>& rs = it->runs;
            for (size_t q = 0; q < rs.size(); q++) {
                const int64_t end = q + 1 < rs.size() ? rs[q + 1].x : m;
                ::memcpy(g->labels_out + rs[q].y, g->h_labels + rs[q].x, 4 * (size_t)(end - rs[q].x));
            }
            g->stats.hits_done += m;
            g->stats.buffers_done++;
            g->label_pool.push_back(it->d_labels);
            g->chunks.erase(it);
        }
        if (nd < cap) break;
    }
    return HC_OK;
}

static int take_slot(hc_ingest* g, int* out)
{
    for (;;) {
        for (int i = 0; i < (int)g->slots.size(); i++)
            if (g->slots[i].state == Slot::kFree) {
                Slot& sl = g->slots[i];
                // the previous use's host-to-device copy must be over before refilling
                hipError_t e = hipEventSynchronize(sl.copied);
                if (e != hipSuccess) return fail_ing(g, HC_ERR_DEVICE, "ingest: copy event");
                sl.state = Slot::kFilling;
                sl.count = 0;
                sl.n_runs = 0;
                *out = i;
                return HC_OK;
            }
        // every buffer is filling or being read: wait for the oldest push to run
        g->stats.waits++;
        int rc = stream_wait_one(g->st);
        if (rc == HC_OK) rc = collect(g);
        if (rc != HC_OK) return rc;
    }
}

static int send(hc_ingest* g, int i)
{
    Slot& sl = g->slots[i];
    if (sl.count == 0) {
        sl.state = Slot::kFree;
        return HC_OK;
    }
    Chunk ch;
    ch.seq = g->seq;
    if (!g->label_pool.empty()) {
        ch.d_labels = g->label_pool.back();
        g->label_pool.pop_back();
    } else if (hipMalloc(&ch.d_labels, 4 * (size_t)g->cfg.buffer_hits) != hipSuccess) {
        return fail_ing(g, HC_ERR_DEVICE, "ingest: hipMalloc(labels)");
    }
    ch.runs.assign(sl.h_runs, sl.h_runs + sl.n_runs);
    ch.count = sl.count;
    hipError_t e = hipMemcpyAsync(sl.d_hits, sl.h_hits, sizeof(hc_hit) * (size_t)sl.count, hipMemcpyHostToDevice,
                                  g->cs);
    // the arrival ids go up as runs and are expanded into per-hit ids there
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_runs, sl.h_runs, sizeof(int2) * (size_t)sl.n_runs, hipMemcpyHostToDevice, g->cs);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_ingest_ids, dim3((unsigned)((sl.count + 255) / 256)), dim3(256), 0, g->cs, sl.d_runs,
                           sl.n_runs, (int32_t)sl.count, sl.d_ids);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(sl.copied, g->cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(g->s, sl.copied, 0);
    if (e != hipSuccess) {
        g->label_pool.push_back(ch.d_labels);
        return fail_ing(g, HC_ERR_DEVICE, "ingest: host-to-device copy");
    }
    sl.push = stream_pushes_enqueued(g->st);
    int rc = hc_stream_push_ids(g->st, sl.d_hits, sl.d_ids, (int32_t)sl.count, ch.d_labels, g->seq);
    if (rc != HC_OK) {
        g->label_pool.push_back(ch.d_labels);
        return fail_ing(g, rc, std::string("ingest: push: ") + hc_last_error());
    }
    sl.state = Slot::kPushed;
    g->chunks.push_back(std::move(ch));
    g->seq++;
    g->stats.buffers_sent++;
    return collect(g);
}

// The arrival ids of hits appended at the buffer's end from id on: they
// extend the last run when they continue it, else open a new one (at most one
// run per hit, so the run arrays of b entries always suffice).
static void add_ids(Slot& sl, int32_t id)
{
    if (sl.n_runs > 0) {
        const int2 last = sl.h_runs[sl.n_runs - 1];
        if (last.y + (sl.count - last.x) == id) return;  // consecutive: the run goes on
    }
    sl.h_runs[sl.n_runs++] = make_int2((int)sl.count, id);
}

static void add(hc_ingest* g, int i, const hc_hit& h, int32_t id)
{
    Slot& sl = g->slots[i];
    sl.h_hits[sl.count] = h;
    add_ids(sl, id);
    sl.count++;
}

extern "C" {

int hc_ingest_create(const hc_ingest_config* cfg, int32_t* labels_out, int64_t labels_cap, hc_ingest** out)
{
    if (!cfg || !out || (labels_cap > 0 && !labels_out) || labels_cap < 0) return set_error(HC_ERR_ARG, "bad ingest arguments");
    *out = nullptr;
    hc_ingest_config c = *cfg;
    if (!c.width) c.width = 256;
    if (!c.height) c.height = 256;
    if (c.buffer_hits <= 0 || c.reserve_hits < 0 || c.reserve_hits >= c.buffer_hits || c.n_buffers < 0 ||
        c.n_buffers == 1 || c.n_buffers == 2 || c.flags || c.reserved || c.width > 65535 || c.height > 65535)
        return set_error(HC_ERR_ARG, "bad ingest configuration (buffer sizes, at least 3 buffers, flags 0)");
    if (!c.n_buffers) c.n_buffers = 4;
    hc_ingest* g = new hc_ingest();
    g->cfg = c;
    g->labels_out = labels_out;
    g->labels_cap = labels_cap;
    g->s = (hipStream_t)c.stream;
    g->tags.resize(256);
    g->status.resize(256);
    hipError_t e;
    int rc = HC_OK;
    if ((e = hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&g->ls, hipStreamNonBlocking)) != hipSuccess)
        rc = set_device_error(e, "hipStreamCreate");
    if (rc == HC_OK) {
        hc_opts o{};
        o.width = c.width;
        o.height = c.height;
        o.disorder_hint = c.disorder_hint;
        o.stream = c.stream;
        rc = hc_stream_create(&o, c.dt, c.max_disorder_ticks, &g->st);
    }
    const size_t b = (size_t)c.buffer_hits;
    g->slots.resize(c.n_buffers);
    for (Slot& sl : g->slots) {
        if (rc != HC_OK) break;
        if ((e = hipHostMalloc((void**)&sl.h_hits, sizeof(hc_hit) * b, hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc((void**)&sl.h_runs, sizeof(int2) * b, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&sl.d_hits, sizeof(hc_hit) * b)) != hipSuccess ||
            (e = hipMalloc(&sl.d_ids, 4 * b)) != hipSuccess ||
            (e = hipMalloc(&sl.d_runs, sizeof(int2) * b)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming)) != hipSuccess)
            rc = set_device_error(e, "ingest buffers");
    }
    if (rc == HC_OK && (e = hipHostMalloc((void**)&g->h_labels, 4 * b, hipHostMallocDefault)) != hipSuccess)
        rc = set_device_error(e, "ingest label staging");
    if (rc == HC_OK) {
        stream_configure(g->st, c.n_buffers - 1, false);
        rc = hc_stream_reserve(g->st, c.buffer_hits);
    }
    if (rc != HC_OK) {
        for (Slot& sl : g->slots) free_slot(sl);
        if (g->h_labels) (void)hipHostFree(g->h_labels);
        if (g->st) hc_stream_destroy(g->st);
        if (g->cs) (void)hipStreamDestroy(g->cs);
        if (g->ls) (void)hipStreamDestroy(g->ls);
        delete g;
        return rc;
    }
    *out = g;
    return HC_OK;
}

int hc_ingest_feed(hc_ingest* g, const hc_hit* hits, int64_t n)
{
    if (!g || n < 0 || (n > 0 && !hits)) return set_error(HC_ERR_ARG, "bad feed arguments");
    if (g->failed) return set_error(HC_ERR_DEVICE, "ingest failed earlier");
    if (g->fed + n > g->labels_cap || g->fed + n > 0x7FFFFFFF)
        return set_error(HC_ERR_OVERFLOW, "more hits than the labels array holds");
    const int64_t b = g->cfg.buffer_hits, bt = g->cfg.reserve_hits;
    const uint64_t tc = g->cfg.t_closing, t = g->cfg.max_disorder_ticks;
    const uint64_t send_gap = ~0ull - t < tc ? ~0ull : t + tc;
    int rc = HC_OK;
    for (int64_t k = 0; k < n; k++) {
        if (g->cur < 0 && (rc = take_slot(g, &g->cur)) != HC_OK) return rc;
        Slot& buf = g->slots[g->cur];
        if (buf.count < b - bt) {
            // first part of the buffer: every hit is taken and toa_max tracked,
            // so a whole run of hits moves in one copy.  No hit of the run can
            // trigger the send below (toa_max already covers it).
            const int64_t m = n - k < (b - bt) - buf.count ? n - k : (b - bt) - buf.count;
            add_ids(buf, (int32_t)g->fed);
            g->toa_max = copy_hits_max(buf.h_hits + buf.count, hits + k, m, g->has_max ? g->toa_max : 0);
            g->has_max = true;
            buf.count += m;
            g->fed += m;
            k += m - 1;
            continue;
        }
        const hc_hit& h = hits[k];
        const int32_t id = (int32_t)(g->fed++);
        if (h.toa < (~0ull - g->toa_max < tc ? ~0ull : g->toa_max + tc) && buf.count < b) {
            add(g, g->cur, h, id);  // may still close a cluster that the buffer holds
        } else {
            if (g->nxt < 0 && (rc = take_slot(g, &g->nxt)) != HC_OK) return rc;
            if (g->slots[g->nxt].count == b) {  // the next buffer is full too: the current one has to go
                g->stats.forced_sends++;
                if ((rc = send(g, g->cur)) != HC_OK) return rc;
                g->cur = g->nxt;
                g->nxt = -1;
                if ((rc = take_slot(g, &g->nxt)) != HC_OK) return rc;
            }
            add(g, g->nxt, h, id);
            g->stats.diverted++;
        }
        // no later hit can belong to the current buffer any more: send it
        if (g->has_max && h.toa > g->toa_max && h.toa - g->toa_max > send_gap && g->cur >= 0) {
            if ((rc = send(g, g->cur)) != HC_OK) return rc;
            g->cur = g->nxt;
            g->nxt = -1;
        }
    }
    g->stats.hits_fed = g->fed;
    return HC_OK;
}

int hc_ingest_finish(hc_ingest* g)
{
    if (!g) return set_error(HC_ERR_ARG, "ingest is NULL");
    if (g->failed) return set_error(HC_ERR_DEVICE, "ingest failed earlier");
    int rc = HC_OK;
    if (g->cur >= 0 && (rc = send(g, g->cur)) != HC_OK) return rc;
    if (g->nxt >= 0 && (rc = send(g, g->nxt)) != HC_OK) return rc;
    g->cur = g->nxt = -1;
    if ((rc = hc_stream_flush(g->st)) != HC_OK) return fail_ing(g, rc, std::string("ingest: ") + hc_last_error());
    if ((rc = collect(g)) != HC_OK) return rc;
    if (!g->chunks.empty()) return fail_ing(g, HC_ERR_DEVICE, "ingest: a buffer never completed");
    g->has_max = false;  // the stream continues as a new segment (see hc_stream_flush)
    return HC_OK;
}

int hc_ingest_stats_read(const hc_ingest* g, hc_ingest_stats* out)
{
    if (!g || !out) return set_error(HC_ERR_ARG, "NULL argument");
    *out = g->stats;
    return HC_OK;
}

void hc_ingest_destroy(hc_ingest* g)
{
    if (!g) return;
    if (g->st) hc_stream_destroy(g->st);
    (void)hipStreamSynchronize(g->cs);
    (void)hipStreamSynchronize(g->ls);
    for (Slot& sl : g->slots) free_slot(sl);
    for (Chunk& ch : g->chunks) (void)hipFree(ch.d_labels);
    for (int32_t* p : g->label_pool) (void)hipFree(p);
    if (g->h_labels) (void)hipHostFree(g->h_labels);
    (void)hipStreamDestroy(g->cs);
    (void)hipStreamDestroy(g->ls);
    delete g;
}

}  // extern "C"
