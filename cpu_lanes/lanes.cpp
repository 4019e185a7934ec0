// Multi-lane CPU clustering of Timepix hits: the paper's CPU method
// (Section 3) as a comparison baseline for the GPU library.  It is not used
// by the GPU library, and it is not the parity oracle.
//
// Temporal splitting (Section 3.2.3): the ToA range is cut into windows of
// equal duration, dealt round-robin to the lanes (one thread each).  A lane
// orders each of its windows by (ToA, index) and clusters it with the
// data-driven sweep (Algorithm "processHit"): a per-pixel matrix holds the
// latest hit seen at every pixel, a hit looks at its own pixel and its eight
// neighbours and joins (union-find, root = the earliest hit, the paper's time
// invariant) every one within dt.  Clusters near a window border -- with a
// hit less than dt from it -- are border clusters (Section 3.3); the merge
// step tests every pair of border clusters of the two sides with the
// paper's cascade: their time distance, then their bounding boxes (grown by
// one pixel, since neighbours may touch), then a full check of the hits
// within dt of the border (the larger side's hits in a per-pixel table, the
// smaller side's looked up at their 9 pixels).  Borders are merged in
// parallel, one lane per border, round-robin.  Labels are the smallest input
// index of each merged cluster, as everywhere in this project.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

struct Hit {
    uint64_t toa;
    uint16_t x, y, tot, reserved;
};

struct Cluster {  // a window-local cluster
    uint64_t t0, t1;            // first and last ToA
    uint16_t x0, x1, y0, y1;    // bounding box
    int32_t min_idx;            // smallest input index
};

int32_t find(std::vector<int32_t>& p, int32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

struct Window {
    std::vector<int64_t> idx;    // input indices of its hits, (ToA, index) order
    std::vector<int32_t> cl;     // per hit: window-local cluster id
    std::vector<Cluster> clusters;
};

struct Shared {
    const Hit* hits;
    int64_t n;
    uint32_t W, H;
    uint64_t dt, tmin, span;
    int64_t n_windows;
    std::vector<Window> win;
};

// Cluster one window with the sweep; the matrix holds, per pixel, the
// latest slot and a stamp of the window that wrote it.
void cluster_window(Shared& S, int64_t w, std::vector<int32_t>& last, std::vector<int64_t>& stamp)
{
    Window& win = S.win[w];
    const int64_t m = (int64_t)win.idx.size();
    std::sort(win.idx.begin(), win.idx.end(), [&](int64_t a, int64_t b) {
        return S.hits[a].toa < S.hits[b].toa || (S.hits[a].toa == S.hits[b].toa && a < b);
    });
    std::vector<int32_t> par(m);
    std::iota(par.begin(), par.end(), 0);
    for (int64_t s = 0; s < m; s++) {
        const Hit& h = S.hits[win.idx[s]];
        for (int dy = -1; dy <= 1; dy++) {
            const int qy = (int)h.y + dy;
            if (qy < 0 || qy >= (int)S.H) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int qx = (int)h.x + dx;
                if (qx < 0 || qx >= (int)S.W) continue;
                const size_t q = (size_t)qy * S.W + (size_t)qx;
                if (stamp[q] != w) continue;
                const int32_t j = last[q];
                if (h.toa - S.hits[win.idx[j]].toa <= S.dt) {
                    const int32_t a = find(par, (int32_t)s), b = find(par, j);
                    if (a != b) par[std::max(a, b)] = std::min(a, b);  // the earlier hit stays the root
                }
            }
        }
        const size_t p = (size_t)h.y * S.W + h.x;
        last[p] = (int32_t)s;
        stamp[p] = w;
    }
    win.cl.assign(m, -1);
    std::vector<int32_t> id(m, -1);
    for (int64_t s = 0; s < m; s++) {
        const int32_t r = find(par, (int32_t)s);
        if (id[r] < 0) {
            id[r] = (int32_t)win.clusters.size();
            const Hit& h = S.hits[win.idx[s]];
            win.clusters.push_back(Cluster{h.toa, h.toa, h.x, h.x, h.y, h.y, (int32_t)win.idx[s]});
        }
        const int32_t c = id[r];
        win.cl[s] = c;
        Cluster& k = win.clusters[c];
        const Hit& h = S.hits[win.idx[s]];
        k.t1 = std::max(k.t1, h.toa);
        k.x0 = std::min(k.x0, h.x);
        k.x1 = std::max(k.x1, h.x);
        k.y0 = std::min(k.y0, h.y);
        k.y1 = std::max(k.y1, h.y);
        k.min_idx = std::min<int32_t>(k.min_idx, (int32_t)win.idx[s]);
    }
}

uint64_t sat_add(uint64_t a, uint64_t b) { return ~0ull - a < b ? ~0ull : a + b; }
uint64_t sat_sub(uint64_t a, uint64_t b) { return a > b ? a - b : 0; }

// Border between window w and the next non-empty window: cluster pairs
// (global ids) that must merge.
void merge_border(Shared& S, int64_t w, int64_t v, const std::vector<int64_t>& base,
                  std::vector<std::pair<int64_t, int64_t>>& out)
{
    const Window& L = S.win[w];
    const Window& R = S.win[v];
    const uint64_t border = S.tmin + (uint64_t)v * S.span;  // the right window's start
    // hits within dt of the border on each side (the only ends of a crossing edge)
    std::vector<int64_t> lh, rh;
    for (int64_t s = (int64_t)L.idx.size() - 1; s >= 0 && S.hits[L.idx[s]].toa >= sat_sub(border, S.dt); s--) lh.push_back(s);
    for (int64_t s = 0; s < (int64_t)R.idx.size() && S.hits[R.idx[s]].toa <= sat_add(border, S.dt); s++) rh.push_back(s);
    if (lh.empty() || rh.empty()) return;
    // border clusters of both sides
    std::vector<int32_t> lc, rc;
    for (int64_t s : lh) lc.push_back(L.cl[s]);
    for (int64_t s : rh) rc.push_back(R.cl[s]);
    std::sort(lc.begin(), lc.end());
    lc.erase(std::unique(lc.begin(), lc.end()), lc.end());
    std::sort(rc.begin(), rc.end());
    rc.erase(std::unique(rc.begin(), rc.end()), rc.end());
    std::unordered_map<int32_t, std::vector<int64_t>> lhits, rhits;
    for (int64_t s : lh) lhits[L.cl[s]].push_back(L.idx[s]);
    for (int64_t s : rh) rhits[R.cl[s]].push_back(R.idx[s]);
    std::unordered_map<uint32_t, std::vector<uint64_t>> table;  // pixel -> ToAs of the larger side
    for (int32_t a : lc) {
        const Cluster& ca = L.clusters[a];
        for (int32_t b : rc) {
            const Cluster& cb = R.clusters[b];
            // 1. time distance of the clusters
            const uint64_t gap = std::max({ca.t0 > cb.t1 ? ca.t0 - cb.t1 : 0, cb.t0 > ca.t1 ? cb.t0 - ca.t1 : 0});
            if (gap > S.dt) continue;
            // 2. bounding boxes, grown by one pixel, must intersect
            if ((int)ca.x1 + 1 < (int)cb.x0 || (int)cb.x1 + 1 < (int)ca.x0 || (int)ca.y1 + 1 < (int)cb.y0 ||
                (int)cb.y1 + 1 < (int)ca.y0)
                continue;
            // 3. full check on the hits near the border
            const std::vector<int64_t>& ha = lhits[a];
            const std::vector<int64_t>& hb = rhits[b];
            const bool a_big = ha.size() >= hb.size();
            const std::vector<int64_t>& big = a_big ? ha : hb;
            const std::vector<int64_t>& small = a_big ? hb : ha;
            table.clear();
            for (int64_t i : big) table[(uint32_t)S.hits[i].y * S.W + S.hits[i].x].push_back(S.hits[i].toa);
            bool joined = false;
            for (int64_t i : small) {
                const Hit& h = S.hits[i];
                for (int dy = -1; dy <= 1 && !joined; dy++) {
                    const int qy = (int)h.y + dy;
                    if (qy < 0 || qy >= (int)S.H) continue;
                    for (int dx = -1; dx <= 1 && !joined; dx++) {
                        const int qx = (int)h.x + dx;
                        if (qx < 0 || qx >= (int)S.W) continue;
                        auto it = table.find((uint32_t)qy * S.W + qx);
                        if (it == table.end()) continue;
                        for (uint64_t t : it->second)
                            if ((t > h.toa ? t - h.toa : h.toa - t) <= S.dt) {
                                joined = true;
                                break;
                            }
                    }
                }
                if (joined) break;
            }
            if (joined) out.emplace_back(base[w] + a, base[v] + b);
        }
    }
}

}  // namespace

extern "C" {

// labels[n]: smallest input index of every hit's cluster (Section 2
// (iii)(a)).  n_lanes threads; windows of `window_ticks` ToA ticks, widened to
// dt + 1 when shorter (the paper takes windows much longer than dt: then an
// edge -- two hits at most dt apart -- crosses at most one border; with
// dt = infinity there is one window).  Returns the number of clusters, or -1
// for bad arguments, -2 for a hit off the sensor.
int64_t lanes_cluster(const void* hits_v, int64_t n, uint32_t W, uint32_t H, uint64_t dt, int n_lanes,
                      uint64_t window_ticks, int32_t* labels)
{
    const Hit* hits = (const Hit*)hits_v;
    if (n < 0 || n > INT32_MAX || W == 0 || H == 0 || n_lanes < 1 || window_ticks == 0 || (n > 0 && !labels))
        return -1;
    if (n == 0) return 0;
    for (int64_t i = 0; i < n; i++)
        if (hits[i].x >= W || hits[i].y >= H) return -2;
    Shared S;
    S.hits = hits;
    S.n = n;
    S.W = W;
    S.H = H;
    S.dt = dt;
    if (window_ticks <= dt) window_ticks = dt == ~0ull ? ~0ull : dt + 1;
    S.span = window_ticks;
    uint64_t tmin = ~0ull, tmax = 0;
    for (int64_t i = 0; i < n; i++) {
        tmin = std::min(tmin, hits[i].toa);
        tmax = std::max(tmax, hits[i].toa);
    }
    S.tmin = tmin;
    S.n_windows = (int64_t)((tmax - tmin) / window_ticks) + 1;
    S.win.resize(S.n_windows);
    // split by window (the input is only partly sorted, so hits are placed
    // by their ToA, not by their position)
    for (int64_t i = 0; i < n; i++) S.win[(hits[i].toa - tmin) / window_ticks].idx.push_back(i);
    // lanes: windows round-robin
    std::vector<std::thread> th;
    for (int l = 0; l < n_lanes; l++)
        th.emplace_back([&S, l, n_lanes]() {
            std::vector<int32_t> last((size_t)S.W * S.H, 0);
            std::vector<int64_t> stamp((size_t)S.W * S.H, -1);
            for (int64_t w = l; w < S.n_windows; w += n_lanes) cluster_window(S, w, last, stamp);
        });
    for (auto& t : th) t.join();
    th.clear();
    // global cluster ids, then the borders in parallel
    std::vector<int64_t> base(S.n_windows + 1, 0);
    for (int64_t w = 0; w < S.n_windows; w++) base[w + 1] = base[w] + (int64_t)S.win[w].clusters.size();
    std::vector<int64_t> next(S.n_windows, -1);  // next non-empty window
    for (int64_t w = S.n_windows - 1, nx = -1; w >= 0; w--) {
        next[w] = nx;
        if (!S.win[w].idx.empty()) nx = w;
    }
    std::vector<std::vector<std::pair<int64_t, int64_t>>> pairs(n_lanes);
    for (int l = 0; l < n_lanes; l++)
        th.emplace_back([&, l]() {
            for (int64_t w = l; w < S.n_windows; w += n_lanes)
                if (!S.win[w].idx.empty() && next[w] >= 0) merge_border(S, w, next[w], base, pairs[l]);
        });
    for (auto& t : th) t.join();
    std::vector<int32_t> par(base[S.n_windows]);
    std::iota(par.begin(), par.end(), 0);
    for (auto& v : pairs)
        for (auto& pr : v) {
            const int32_t a = find(par, (int32_t)pr.first), b = find(par, (int32_t)pr.second);
            if (a != b) par[std::max(a, b)] = std::min(a, b);
        }
    std::vector<int32_t> mn(base[S.n_windows], INT32_MAX);
    for (int64_t w = 0; w < S.n_windows; w++)
        for (size_t c = 0; c < S.win[w].clusters.size(); c++) {
            const int32_t r = find(par, (int32_t)(base[w] + c));
            mn[r] = std::min(mn[r], S.win[w].clusters[c].min_idx);
        }
    int64_t k = 0;
    for (int64_t g = 0; g < base[S.n_windows]; g++) k += find(par, (int32_t)g) == g;
    for (int64_t w = 0; w < S.n_windows; w++) {
        const Window& win = S.win[w];
        for (size_t s = 0; s < win.idx.size(); s++) labels[win.idx[s]] = mn[find(par, (int32_t)(base[w] + win.cl[s]))];
    }
    return k;
}

}  // extern "C"
