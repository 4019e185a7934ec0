// Served form: a request loop over many detector streams with continuous
// batching.  Each stream has a host worker thread, a HIP stream and an
// hc_stream (open clusters stay on the device and are stitched exactly across
// chunks).  Chunks wait per stream in arrival order and are admitted when a
// device slot is free and the memory they need fits the HBM budget; admitted
// chunks of different streams run concurrently on the device, and a stream's
// own chunks are pipelined: pushes are asynchronous, so the worker copies and
// enqueues the next push while earlier ones still run, and retires pushes
// (slot release, processing stamp, closed clusters to the host) as their
// completion is observed.  Chunks of one stream that are queued together are
// merged into one push (up to the reserved chunk size), each still accepted
// or rejected on its own: a push has a fixed cost of some tens of kernels,
// which small chunks would otherwise pay one by one.  Final labels go back on
// a separate copy stream, which never waits for pushes still in flight.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hc_internal.h"

using namespace hc;

namespace {

constexpr size_t kMinBlock = 64 << 10;
constexpr int kServerDepth = 2;  // pushes in flight per stream

size_t block_class(size_t bytes)
{
    size_t c = kMinBlock;
    while (c < bytes) c <<= 1;
    return c;
}

struct Req {
    bool flush;
    uint64_t tag;
    const hc_hit* hits;
    int32_t n;
    int32_t* labels;
    uint64_t t_arrive;
};

struct Pending {
    uint64_t tag;
    int32_t n;
    int32_t n_closed;
    int32_t* labels_host;
    void* labels_dev;
    size_t labels_class;
    uint64_t t_arrive, t_admit, t_processed;
};

struct StreamCtx {
    int id = 0;
    hc_stream* st = nullptr;
    hipStream_t hs = nullptr;  // hits in, pushes
    hipStream_t cs = nullptr;  // final labels out
    std::thread th;
    std::condition_variable cv;
    std::deque<Req> q;                           // guarded by the server mutex
    std::mutex cmu;                              // guards closed / closed_head
    std::deque<std::vector<hc_features>> closed; // closed-cluster features, one block per drain
    size_t closed_head = 0;                      // rows of closed.front() already handed out
    std::vector<std::vector<hc_features>> spare; // blocks read out by the caller, for reuse
    std::unordered_map<uint64_t, Pending> pend;  // worker-only, keyed by internal sequence number
    uint64_t seq = 0;
    int in_device = 0;                           // pushed chunks not yet retired (worker-only)
    void* hits_dev = nullptr;
    size_t hits_bytes = 0;
    size_t state_bytes = 0;  // device bytes of the hc_stream counted in `used`
    uint64_t* tags_pin = nullptr;      // pinned drain buffers (finished chunk tags,
    int32_t* status_pin = nullptr;     // their status,
    hc_features* feats_pin = nullptr;  // closed-cluster features)
    std::vector<RetiredPush> retired;  // scratch
};

constexpr int kDrainTags = 256, kDrainFeats = 1 << 16;
constexpr size_t kSpareBlocks = 8;  // read-out closed-feature blocks kept per stream for reuse

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

uint64_t quantile(std::vector<uint64_t> v, double q)
{
    if (v.empty()) return 0;
    const size_t k = (size_t)(q * (double)(v.size() - 1) + 0.5);
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
}

}  // namespace

struct hc_server {
    hc_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable budget_cv, idle_cv;
    uint64_t used = 0, peak = 0, progress = 0;
    int slots_used = 0, peak_slots = 0;
    int64_t submitted = 0, completed = 0, rejected = 0, hits_completed = 0, queued = 0, pending_final = 0;
    int64_t pushes = 0;  // device pushes enqueued
    int working = 0;  // requests taken by a worker and not yet through their device processing
    std::atomic<uint64_t> ns_admit{0}, ns_push{0}, ns_drain{0}, ns_final{0};
    bool stopping = false;
    std::vector<StreamCtx*> streams;
    std::deque<hc_completion> done;
    std::vector<uint64_t> lat_proc, lat_final;
    std::map<size_t, std::vector<void*>> free_blocks;  // label buffers ready for reuse (counted in used)

    void account(int64_t delta)
    {
        used = (uint64_t)((int64_t)used + delta);
        if (used > peak) peak = used;
    }

    // Release cached label blocks (lock held); returns bytes freed.
    uint64_t trim_cache()
    {
        uint64_t freed = 0;
        for (auto& kv : free_blocks)
            for (void* p : kv.second) {
                (void)hipFree(p);
                freed += kv.first;
            }
        free_blocks.clear();
        account(-(int64_t)freed);
        return freed;
    }

    void complete(const hc_completion& c)
    {
        done.push_back(c);
        completed++;
        if (c.status == HC_OK) {
            hits_completed += c.n_hits;
            lat_final.push_back(c.t_final_ns - c.t_arrive_ns);
        } else {
            rejected++;
        }
        progress++;
        budget_cv.notify_all();
    }

    void worker(StreamCtx* cx);
    bool try_admit(StreamCtx* cx, const Req& r, Pending* p, size_t* hits_need, uint64_t* charged);
    bool try_admit_more(StreamCtx* cx, const Req& r, int64_t hits_before, Pending* p, size_t* hits_need,
                        uint64_t* charged);
    void run_push(StreamCtx* cx, std::vector<Req>& rs, std::vector<Pending>& ps, size_t hits_need,
                  uint64_t charged);
    void advance(StreamCtx* cx);
    void finish(StreamCtx* cx, uint64_t seq, int32_t status);
};

// A chunk is done: final labels to the caller (or its rejection), then its
// completion record.
void hc_server::finish(StreamCtx* cx, uint64_t seq, int32_t status)
{
    auto it = cx->pend.find(seq);
    if (it == cx->pend.end()) return;
    Pending p = it->second;
    cx->pend.erase(it);
    const uint64_t f0 = now_ns();
    if (status == HC_OK && p.n > 0) {
        hipError_t e = hipMemcpyAsync(p.labels_host, p.labels_dev, 4 * (size_t)p.n, hipMemcpyDeviceToHost, cx->cs);
        if (e == hipSuccess) e = hipStreamSynchronize(cx->cs);
        if (e != hipSuccess) status = set_device_error(e, "server: label copy");
    }
    hc_completion c{};
    c.tag = p.tag;
    c.stream_id = cx->id;
    c.status = status;
    c.n_hits = p.n;
    c.n_closed = status == HC_OK ? p.n_closed : 0;
    c.t_arrive_ns = p.t_arrive;
    c.t_admit_ns = p.t_admit;
    c.t_processed_ns = p.t_processed ? p.t_processed : now_ns();
    c.t_final_ns = now_ns();
    ns_final += c.t_final_ns - f0;
    std::lock_guard<std::mutex> lk(mu);
    if (p.labels_dev) free_blocks[p.labels_class].push_back(p.labels_dev);
    pending_final--;
    complete(c);
}

// Retire the pushes that completed: closed clusters to the host, processing
// stamps, slots released; then the chunks that finished.
void hc_server::advance(StreamCtx* cx)
{
    cx->retired.clear();
    stream_take_retired(cx->st, &cx->retired);
    std::vector<std::pair<uint64_t, int32_t>> fin;
    const uint64_t dr0 = now_ns();
    for (;;) {
        int32_t nd = 0, nc = 0;
        if (hc_stream_poll(cx->st, cx->tags_pin, cx->status_pin, kDrainTags, &nd, cx->feats_pin, kDrainFeats, &nc) !=
            HC_OK)
            break;
        if (nc > 0) {  // copied outside any lock; only the hand-overs are guarded
            // a block the caller has read out is reused: fresh host memory
            // costs a page fault per 4 KiB on first touch, far more than the copy
            std::vector<hc_features> blk;
            {
                std::lock_guard<std::mutex> lk(cx->cmu);
                if (!cx->spare.empty()) {
                    blk = std::move(cx->spare.back());
                    cx->spare.pop_back();
                }
            }
            if (blk.capacity() < (size_t)kDrainFeats) blk.reserve(kDrainFeats);
            blk.assign(cx->feats_pin, cx->feats_pin + nc);
            std::lock_guard<std::mutex> lk(cx->cmu);
            cx->closed.push_back(std::move(blk));
        }
        for (int32_t k = 0; k < nd; k++) fin.emplace_back(cx->tags_pin[k], cx->status_pin[k]);
        if (nd < kDrainTags && nc < kDrainFeats) break;
    }
    const uint64_t tp = now_ns();
    if (!cx->retired.empty() || !fin.empty()) ns_drain += tp - dr0;
    if (!cx->retired.empty()) {
        const size_t state_now = stream_device_bytes(cx->st);
        std::lock_guard<std::mutex> lk(mu);
        for (const RetiredPush& r : cx->retired) {
            auto it = cx->pend.find(r.tag);
            if (it != cx->pend.end()) {
                it->second.t_processed = tp;
                it->second.n_closed = r.n_closed;
                lat_proc.push_back(tp - it->second.t_arrive);
            }
            working--;
            if (r.last) {  // one slot per push
                slots_used--;
                cx->in_device--;
            }
        }
        account((int64_t)state_now - (int64_t)cx->state_bytes);
        cx->state_bytes = state_now;
        progress++;
        budget_cv.notify_all();
        idle_cv.notify_all();
    }
    for (const auto& f : fin) finish(cx, f.first, f.second);
}

// Admission (lock held): a free slot and the memory of this push within the
// budget.  On success the memory is charged and *p holds the label block.
bool hc_server::try_admit(StreamCtx* cx, const Req& r, Pending* p, size_t* hits_need, uint64_t* charged)
{
    *hits_need = r.n > 0 ? block_class(sizeof(hc_hit) * (size_t)r.n) : 0;
    const size_t hits_grow = *hits_need > cx->hits_bytes ? *hits_need - cx->hits_bytes : 0;
    size_t transient = 0;
    const size_t after = r.n > 0 ? stream_bytes_after_push(cx->st, r.n, &transient) : cx->state_bytes;
    const size_t state_grow = after > cx->state_bytes ? after - cx->state_bytes : 0;
    p->labels_class = r.n > 0 ? block_class(4 * (size_t)r.n) : 0;
    auto fb = free_blocks.lower_bound(p->labels_class);
    while (fb != free_blocks.end() && fb->second.empty()) ++fb;
    const bool reuse = r.n > 0 && fb != free_blocks.end();
    const uint64_t need = hits_grow + state_grow + transient + (reuse || r.n == 0 ? 0 : p->labels_class);
    if (slots_used >= cfg.max_slots || used + need > cfg.hbm_budget) {
        if (used + need > cfg.hbm_budget && !free_blocks.empty() && trim_cache() > 0)
            return try_admit(cx, r, p, hits_need, charged);
        return false;
    }
    if (reuse) {
        p->labels_dev = fb->second.back();
        p->labels_class = fb->first;
        fb->second.pop_back();
    }
    account((int64_t)need);
    *charged = need - (reuse || r.n == 0 ? 0 : p->labels_class) - hits_grow;  // the stream's share
    slots_used++;
    peak_slots = std::max(peak_slots, slots_used);
    queued--;
    progress++;
    return true;
}

// Admission of one more queued chunk into the push being formed (lock held):
// no slot of its own, only the memory it adds (the push's hits, its labels,
// the stream state for the larger push) within the budget.
bool hc_server::try_admit_more(StreamCtx* cx, const Req& r, int64_t hits_before, Pending* p, size_t* hits_need,
                               uint64_t* charged)
{
    const size_t need_h = block_class(sizeof(hc_hit) * (size_t)(hits_before + r.n));
    const size_t held_h = std::max(*hits_need, cx->hits_bytes);
    const size_t hits_grow = need_h > held_h ? need_h - held_h : 0;
    size_t tr0 = 0, tr1 = 0;
    const size_t s0 = stream_bytes_after_push(cx->st, hits_before, &tr0);
    const size_t s1 = stream_bytes_after_push(cx->st, hits_before + r.n, &tr1);
    const size_t state_grow = (s1 > s0 ? s1 - s0 : 0) + (tr1 > tr0 ? tr1 - tr0 : 0);
    p->labels_class = block_class(4 * (size_t)r.n);
    auto fb = free_blocks.lower_bound(p->labels_class);
    while (fb != free_blocks.end() && fb->second.empty()) ++fb;
    const bool reuse = fb != free_blocks.end();
    const uint64_t need = hits_grow + state_grow + (reuse ? 0 : p->labels_class);
    if (used + need > cfg.hbm_budget) return false;
    if (reuse) {
        p->labels_dev = fb->second.back();
        p->labels_class = fb->first;
        fb->second.pop_back();
    }
    account((int64_t)need);
    *hits_need = std::max(*hits_need, need_h);
    *charged += state_grow;  // the stream's share, reconciled after the push
    queued--;
    return true;
}

// One push of the admitted chunks rs (one stream, in order, none empty
// unless it is alone): hits copied in behind each other, labels blocks,
// one hc_stream push, and each chunk pending until its labels are final.
void hc_server::run_push(StreamCtx* cx, std::vector<Req>& rs, std::vector<Pending>& ps, size_t hits_need,
                         uint64_t charged)
{
    const int k = (int)rs.size();
    hipError_t e = hipSuccess;
    int rc = HC_OK;
    if (hits_need > cx->hits_bytes) {
        // pushes in flight may still read the old buffer
        if ((e = hipStreamSynchronize(cx->hs)) != hipSuccess) rc = set_device_error(e, "server: hits buffer");
        (void)hipFree(cx->hits_dev);
        cx->hits_dev = nullptr;
        const size_t grow = hits_need - cx->hits_bytes;
        if (rc == HC_OK && (e = hipMalloc(&cx->hits_dev, hits_need)) != hipSuccess) {
            cx->hits_dev = nullptr;
            rc = set_device_error(e, "server: hits buffer");
        }
        if (rc == HC_OK) {
            cx->hits_bytes = hits_need;
        } else {
            std::lock_guard<std::mutex> lk(mu);
            account(-(int64_t)cx->hits_bytes - (int64_t)grow);
            cx->hits_bytes = 0;
        }
    }
    int64_t total = 0;
    for (int j = 0; j < k; j++) total += rs[j].n;
    for (int j = 0; j < k && rc == HC_OK; j++)
        if (rs[j].n > 0 && !ps[j].labels_dev) {
            if ((e = hipMalloc(&ps[j].labels_dev, ps[j].labels_class)) != hipSuccess) {
                ps[j].labels_dev = nullptr;
                rc = set_device_error(e, "server: labels buffer");
            }
        }
    // the hits buffer is rewritten only behind the earlier pushes on the same
    // stream; chunks that lie back to back in host memory go in one copy
    for (int j = 0, at = 0; j < k && rc == HC_OK;) {
        int j1 = j + 1;
        int64_t m = rs[j].n;
        while (j1 < k && rs[j1].hits == rs[j1 - 1].hits + rs[j1 - 1].n) m += rs[j1++].n;
        if (m > 0 && (e = hipMemcpyAsync((hc_hit*)cx->hits_dev + at, rs[j].hits, sizeof(hc_hit) * (size_t)m,
                                         hipMemcpyHostToDevice, cx->hs)) != hipSuccess)
            rc = set_device_error(e, "server: hits copy");
        at += (int)m;
        j = j1;
    }
    std::vector<uint64_t> seqs(k);
    for (int j = 0; j < k; j++) seqs[j] = cx->seq++;
    if (rc == HC_OK && total > 0) {
        int32_t counts[kMaxPushChunks];
        int32_t* labs[kMaxPushChunks];
        for (int j = 0; j < k; j++) {
            counts[j] = rs[j].n;
            labs[j] = (int32_t*)ps[j].labels_dev;
        }
        rc = hc_stream_push_chunks(cx->st, (const hc_hit*)cx->hits_dev, k, counts, labs, seqs.data());
    }
    const uint64_t d0 = now_ns();
    ns_push += d0 - ps[0].t_admit;
    const size_t state_now = stream_device_bytes(cx->st);
    std::lock_guard<std::mutex> lk(mu);
    // the growth charged at admission becomes the stream's actual size
    account((int64_t)state_now - (int64_t)cx->state_bytes - (int64_t)charged);
    cx->state_bytes = state_now;
    if (rc != HC_OK || total == 0) {  // nothing runs: every chunk is done at once
        slots_used--;
        for (int j = 0; j < k; j++) {
            working--;
            hc_completion c{};
            c.tag = rs[j].tag;
            c.stream_id = cx->id;
            c.status = rc;
            c.n_hits = rs[j].n;
            c.t_arrive_ns = rs[j].t_arrive;
            c.t_admit_ns = ps[j].t_admit;
            c.t_processed_ns = c.t_final_ns = now_ns();
            if (rc == HC_OK) lat_proc.push_back(c.t_processed_ns - rs[j].t_arrive);
            if (ps[j].labels_dev) free_blocks[ps[j].labels_class].push_back(ps[j].labels_dev);
            else if (rc != HC_OK && rs[j].n > 0) account(-(int64_t)ps[j].labels_class);  // its block never came
            complete(c);
        }
        idle_cv.notify_all();
        return;
    }
    pushes++;
    cx->in_device++;
    for (int j = 0; j < k; j++) {
        pending_final++;
        cx->pend.emplace(seqs[j], ps[j]);
    }
}

void hc_server::worker(StreamCtx* cx)
{
    (void)hipSetDevice(device);
    for (;;) {
        advance(cx);
        Req r{};
        Pending p{};
        size_t hits_need = 0;
        uint64_t charged = 0;
        bool have = false, flush = false, wait_device = false;
        std::vector<Req> rs;
        std::vector<Pending> ps;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!cx->q.empty()) {
                const Req& front = cx->q.front();
                if (front.flush) {
                    if (cx->in_device == 0) {  // behind every chunk queued before it
                        r = front;
                        cx->q.pop_front();
                        queued--;
                        working++;
                        have = flush = true;
                    } else {
                        wait_device = true;
                    }
                } else {
                    p = Pending{front.tag, front.n, 0, front.labels, nullptr, 0, front.t_arrive, 0, 0};
                    const uint64_t a0 = now_ns();
                    if (try_admit(cx, front, &p, &hits_need, &charged)) {
                        r = front;
                        cx->q.pop_front();
                        working++;
                        have = true;
                        p.t_admit = now_ns();
                        ns_admit += p.t_admit - a0;
                    } else if (cx->in_device > 0) {
                        wait_device = true;  // our own pushes will free a slot or memory
                    } else {
                        const uint64_t p0 = progress;
                        budget_cv.wait_for(lk, std::chrono::milliseconds(200));
                        size_t hn;
                        uint64_t ch;
                        Pending probe = p;
                        if (progress == p0 && slots_used == 0 && !stopping) {
                            // nothing in flight can release memory: this chunk can never fit
                            const uint64_t a1 = now_ns();
                            if (!try_admit(cx, front, &probe, &hn, &ch)) {
                                hc_completion c{};
                                c.tag = front.tag;
                                c.stream_id = cx->id;
                                c.status = HC_ERR_BUDGET;
                                c.n_hits = front.n;
                                c.t_arrive_ns = front.t_arrive;
                                c.t_admit_ns = c.t_processed_ns = c.t_final_ns = a1;
                                cx->q.pop_front();
                                queued--;
                                complete(c);
                                idle_cv.notify_all();
                                continue;
                            }
                            r = front;
                            p = probe;
                            hits_need = hn;
                            charged = ch;
                            cx->q.pop_front();
                            working++;
                            have = true;
                            p.t_admit = now_ns();
                        }
                    }
                }
            } else if (cx->in_device > 0) {
                wait_device = true;
            } else if (stopping) {
                break;  // chunks still waiting for finality are released by hc_server_destroy
            } else if (!cx->pend.empty()) {
                // only finality pending: it needs more data or a flush
                cx->cv.wait_for(lk, std::chrono::milliseconds(50));
            } else {
                cx->cv.wait(lk, [&] { return stopping || !cx->q.empty(); });
            }
            if (have && !flush) {
                // the chunks queued behind it join its push while they fit
                rs.push_back(r);
                ps.push_back(p);
                int64_t total = r.n;
                while (r.n > 0 && (int)rs.size() < kMaxPushChunks && !cx->q.empty()) {
                    const Req& nx = cx->q.front();
                    if (nx.flush || nx.n == 0 || total + nx.n > cfg.max_chunk_hits) break;
                    Pending pn{nx.tag, nx.n, 0, nx.labels, nullptr, 0, nx.t_arrive, 0, 0};
                    if (!try_admit_more(cx, nx, total, &pn, &hits_need, &charged)) break;
                    pn.t_admit = now_ns();
                    rs.push_back(nx);
                    ps.push_back(pn);
                    cx->q.pop_front();
                    working++;
                    total += nx.n;
                }
            }
        }
        try {
            if (have && flush) {
                if (hc_stream_flush(cx->st) != HC_OK) (void)hc_last_error();
                advance(cx);
                std::lock_guard<std::mutex> lk(mu);
                working--;
                progress++;
                idle_cv.notify_all();
                budget_cv.notify_all();
            } else if (have) {
                run_push(cx, rs, ps, hits_need, charged);
            } else if (wait_device) {
                (void)stream_wait_one(cx->st);
            }
        } catch (...) {
            (void)set_error(HC_ERR_DEVICE, "server worker: host exception");
        }
    }
}

extern "C" {

uint64_t hc_server_now_ns(void) { return now_ns(); }

int hc_server_create(const hc_server_config* cfg, hc_server** out)
{
    if (!out || !cfg) return set_error(HC_ERR_ARG, "NULL config or out");
    *out = nullptr;
    hc_server_config c = *cfg;
    if (!c.width) c.width = 256;
    if (!c.height) c.height = 256;
    if (c.width > 65535 || c.height > 65535 || c.flags || c.reserved || c.n_streams < 1 || c.n_streams > 256 ||
        c.max_slots < 0 || c.max_chunk_hits < 0)
        return set_error(HC_ERR_ARG, "bad server configuration");
    if (!c.max_chunk_hits) c.max_chunk_hits = 1 << 20;
    if (!c.max_slots) c.max_slots = kServerDepth * c.n_streams;
    if (!c.hbm_budget) c.hbm_budget = 16ull << 30;
    if (!c.disorder_hint) c.disorder_hint = 4096;
    hc_server* s = new hc_server();
    s->cfg = c;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return set_device_error(e, "hipGetDevice");
    }
    int rc = HC_OK;
    for (int i = 0; i < c.n_streams && rc == HC_OK; i++) {
        StreamCtx* cx = new StreamCtx();
        cx->id = i;
        s->streams.push_back(cx);
        if ((e = hipStreamCreateWithFlags(&cx->hs, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipStreamCreateWithFlags(&cx->cs, hipStreamNonBlocking)) != hipSuccess) {
            rc = set_device_error(e, "hipStreamCreate");
            break;
        }
        hc_opts o{};
        o.width = c.width;
        o.height = c.height;
        o.disorder_hint = c.disorder_hint;
        o.stream = cx->hs;
        if ((rc = hc_stream_create(&o, c.dt, c.max_disorder_ticks, &cx->st)) != HC_OK) break;
        stream_configure(cx->st, kServerDepth, true);
        // everything a chunk of max_chunk_hits needs, allocated once
        if ((rc = hc_stream_reserve(cx->st, c.max_chunk_hits)) != HC_OK) break;
        cx->state_bytes = stream_device_bytes(cx->st);
        s->account((int64_t)cx->state_bytes);
        cx->hits_bytes = block_class(sizeof(hc_hit) * (size_t)c.max_chunk_hits);
        if ((e = hipMalloc(&cx->hits_dev, cx->hits_bytes)) != hipSuccess) {
            cx->hits_bytes = 0;
            rc = set_device_error(e, "hipMalloc(server hits)");
            break;
        }
        s->account((int64_t)cx->hits_bytes);
        if ((e = hipHostMalloc((void**)&cx->tags_pin, sizeof(uint64_t) * kDrainTags, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&cx->status_pin, sizeof(int32_t) * kDrainTags, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&cx->feats_pin, sizeof(hc_features) * kDrainFeats, hipHostMallocDefault)) !=
                hipSuccess) {
            rc = set_device_error(e, "hipHostMalloc(server drain)");
            break;
        }
        // label blocks per stream: the chunks in flight and one awaiting finality
        const size_t lc = block_class(4 * (size_t)c.max_chunk_hits);
        for (int b = 0; b < kServerDepth + 1 && rc == HC_OK; b++) {
            void* p = nullptr;
            if ((e = hipMalloc(&p, lc)) != hipSuccess) {
                rc = set_device_error(e, "hipMalloc(server labels)");
                break;
            }
            s->free_blocks[lc].push_back(p);
            s->account((int64_t)lc);
        }
        if (rc != HC_OK) break;
        if (s->used > c.hbm_budget) {
            rc = set_error(HC_ERR_BUDGET, "budget below the streams' reserved state");
            break;
        }
    }
    if (rc != HC_OK) {
        for (auto& kv : s->free_blocks)
            for (void* p : kv.second) (void)hipFree(p);
        for (StreamCtx* cx : s->streams) {
            if (cx->st) hc_stream_destroy(cx->st);
            (void)hipFree(cx->hits_dev);
            if (cx->tags_pin) (void)hipHostFree(cx->tags_pin);
            if (cx->status_pin) (void)hipHostFree(cx->status_pin);
            if (cx->feats_pin) (void)hipHostFree(cx->feats_pin);
            if (cx->hs) (void)hipStreamDestroy(cx->hs);
            if (cx->cs) (void)hipStreamDestroy(cx->cs);
            delete cx;
        }
        delete s;
        return rc;
    }
    for (StreamCtx* cx : s->streams) cx->th = std::thread([s, cx] { s->worker(cx); });
    *out = s;
    return HC_OK;
}

int hc_server_submit(hc_server* s, int32_t stream_id, const hc_hit* hits, int32_t n, int32_t* labels, uint64_t tag,
                     uint64_t t_arrive_ns)
{
    if (!s || stream_id < 0 || stream_id >= s->cfg.n_streams) return set_error(HC_ERR_ARG, "bad server or stream id");
    if (n < 0 || (n > 0 && (!hits || !labels))) return set_error(HC_ERR_ARG, "bad chunk arguments");
    if (block_class(sizeof(hc_hit) * (size_t)n) + block_class(4 * (size_t)n) > s->cfg.hbm_budget)
        return set_error(HC_ERR_BUDGET, "chunk larger than the memory budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return set_error(HC_ERR_BUSY, "server is shutting down");
    StreamCtx* cx = s->streams[stream_id];
    cx->q.push_back(Req{false, tag, hits, n, labels, t_arrive_ns});
    s->submitted++;
    s->queued++;
    cx->cv.notify_one();
    return HC_OK;
}

int hc_server_flush(hc_server* s, int32_t stream_id)
{
    if (!s || stream_id < 0 || stream_id >= s->cfg.n_streams) return set_error(HC_ERR_ARG, "bad server or stream id");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return set_error(HC_ERR_BUSY, "server is shutting down");
    StreamCtx* cx = s->streams[stream_id];
    cx->q.push_back(Req{true, 0, nullptr, 0, nullptr, 0});
    s->queued++;
    cx->cv.notify_one();
    return HC_OK;
}

int hc_server_poll(hc_server* s, hc_completion* out, int32_t cap, int32_t* n_out)
{
    if (!s || !n_out || (cap > 0 && !out)) return set_error(HC_ERR_ARG, "bad poll arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    return HC_OK;
}

int hc_server_closed(hc_server* s, int32_t stream_id, hc_features* out, int32_t cap, int32_t* n_out)
{
    if (!s || !n_out || stream_id < 0 || stream_id >= s->cfg.n_streams || (cap > 0 && !out))
        return set_error(HC_ERR_ARG, "bad arguments");
    StreamCtx* cx = s->streams[stream_id];
    std::lock_guard<std::mutex> lk(cx->cmu);
    int32_t k = 0;
    while (k < cap && !cx->closed.empty()) {
        const std::vector<hc_features>& blk = cx->closed.front();
        const size_t take = std::min<size_t>((size_t)(cap - k), blk.size() - cx->closed_head);
        ::memcpy(out + k, blk.data() + cx->closed_head, sizeof(hc_features) * take);
        k += (int32_t)take;
        cx->closed_head += take;
        if (cx->closed_head == blk.size()) {
            if (cx->spare.size() < kSpareBlocks) cx->spare.push_back(std::move(cx->closed.front()));
            cx->closed.pop_front();
            cx->closed_head = 0;
        }
    }
    *n_out = k;
    return HC_OK;
}

int hc_server_wait_idle(hc_server* s, int32_t timeout_ms)
{
    if (!s) return set_error(HC_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->idle_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms),
                                        [&] { return s->queued == 0 && s->working == 0; });
    return ok ? HC_OK : set_error(HC_ERR_BUSY, "server still busy");
}

int hc_server_stats_read(hc_server* s, hc_server_stats* out)
{
    if (!s || !out) return set_error(HC_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    hc_server_stats st{};
    st.submitted = s->submitted;
    st.completed = s->completed;
    st.rejected = s->rejected;
    st.hits_completed = s->hits_completed;
    st.queued = s->queued;
    st.pending_final = s->pending_final;
    st.hbm_budget = s->cfg.hbm_budget;
    st.hbm_in_use = s->used;
    st.hbm_peak = s->peak;
    st.max_slots = s->cfg.max_slots;
    st.peak_slots_in_use = s->peak_slots;
    st.processing_p50 = quantile(s->lat_proc, 0.50);
    st.processing_p99 = quantile(s->lat_proc, 0.99);
    st.final_p50 = quantile(s->lat_final, 0.50);
    st.final_p99 = quantile(s->lat_final, 0.99);
    st.ns_admit_wait = s->ns_admit;
    st.ns_push = s->ns_push;
    st.ns_drain = s->ns_drain;
    st.ns_final = s->ns_final;
    st.pushes = s->pushes;
    *out = st;
    return HC_OK;
}

void hc_server_destroy(hc_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (StreamCtx* cx : s->streams) cx->cv.notify_all();
        s->budget_cv.notify_all();
    }
    for (StreamCtx* cx : s->streams)
        if (cx->th.joinable()) cx->th.join();
    for (StreamCtx* cx : s->streams) {
        (void)hipStreamSynchronize(cx->hs);
        (void)hipStreamSynchronize(cx->cs);
        for (auto& kv : cx->pend)
            if (kv.second.labels_dev) (void)hipFree(kv.second.labels_dev);
        hc_stream_destroy(cx->st);
        (void)hipFree(cx->hits_dev);
        (void)hipHostFree(cx->tags_pin);
        (void)hipHostFree(cx->status_pin);
        (void)hipHostFree(cx->feats_pin);
        (void)hipStreamDestroy(cx->hs);
        (void)hipStreamDestroy(cx->cs);
        delete cx;
    }
    for (auto& kv : s->free_blocks)
        for (void* p : kv.second) (void)hipFree(p);
    delete s;
}

}  // extern "C"
