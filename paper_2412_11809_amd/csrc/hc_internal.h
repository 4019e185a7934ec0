// Internal declarations of the hit-clustering library: workspace layout,
// launch parameters and the kernel launchers of each translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "hc.h"

namespace hc {

// ---------------------------------------------------------------- constants
constexpr int kSortThreads = 512;     // threads of the tile-sort / merge kernels
constexpr int kLinkTile = 1024;       // sorted hits per link work-group
constexpr int kLinkHaloCap = 1024;    // earlier hits a link work-group can hold
constexpr uint32_t kLinkWindowMaxDim = 16384;  // window scan: coordinates fit 14 bits
constexpr int kLinkThreads = 512;


constexpr int kFeatTile = 512;        // sorted hits per feature work-group
constexpr int kFeatThreads = 256;
constexpr int kFeatHash = 512;        // root hash slots (>= tile: a tile never fills it)
constexpr int kScanBlock = 2048;      // input indices per compaction block
constexpr int kScanThreads = 256;
constexpr int kFbBlock = 2048;        // elements per fallback radix block
constexpr int kFbThreads = 512;
constexpr int kFbMaxPasses = 8;       // 8-bit digits of a 64-bit key
constexpr int kFbScanSeg = 16384;     // digit counters per parallel scan task
constexpr int kFbGroup = 32;          // blocks per histogram / scatter task (fewer cross-XCD fences)
constexpr int kMaxNeighbourTiles = 64; // sort merge looks at most this far (tiles apart in ToA cost one check)

// Partial or final integer features of one cluster (64 bytes).
struct SlotRec {
    uint32_t size;
    int32_t root;  // carries: the cluster's label; slots: unused
    uint64_t sum_tot, toa_min, toa_max, sum_xt, sum_yt, sum_x, sum_y;
};
static_assert(sizeof(SlotRec) == 64, "slot record is one cache line");

constexpr int kTileQ = 16;  // parts of a sorted tile described by their last key

struct TileInfo {
    uint64_t base;     // smallest ToA in the tile
    uint64_t max_toa;  // largest ToA
    int32_t min_idx;   // input index of the tile's first element in (toa, idx) order
    int32_t max_idx;   // ... and of its last element
    int32_t wide;      // ToA range does not fit 32 bits (tile left unsorted)
    int32_t count;
};

// State of one ticketed fallback radix sort (see hc_radix.h).
struct RadixState {
    int32_t ticket;
    int32_t plan_done;
    int32_t total_tasks;
    int32_t passes;
    int32_t active;
    int32_t pad_;
    uint64_t key_min;
    int32_t hist_done[kFbMaxPasses];
    int32_t scan_done[kFbMaxPasses];
    int32_t scatter_done[kFbMaxPasses];
    int32_t query_done;
    int32_t shift;          // batch sort: chunk id sits above this many ToA bits
    int32_t seg_done[kFbMaxPasses];  // segments of the counter scan finished
    int32_t n_eff;          // elements sorted (the plan may take fewer than count())
    int32_t pad2_[5];
};

struct Status {
    int32_t err_range;      // a hit lies outside the sensor
    int32_t sort_fallback;  // tile sort/merge could not order the input
    int32_t n_overflow;     // link tiles whose halo did not fit
    int32_t n_deep;         // of those, tiles whose halo did not fit the wide kernel either
    int32_t unused_[2];
    int32_t err_internal;   // an index derived from device data was out of range
    int32_t err_span;       // batch sort fallback: a chunk's ToA span too large
    int32_t pad_[8];
    RadixState rs[2];       // [0]: ToA sort fallback, [1]: pixel sort fallback
};

// One independently clustered chunk of the input (the batch form has many;
// the plain path has one).  Tiles of every kind never straddle two chunks:
// the chunk's tiles of kind k are tile0[k] .. tile0[k] + ceil(count / size_k) - 1.
enum TileKind { kSortKind = 0, kLinkKind = 1, kFeatKind = 2, kScanKind = 3 };
struct SegInfo {
    int64_t start;     // first hit (position in the concatenated input)
    int32_t count;
    int32_t pad_;
    uint64_t dt;       // time window of the chunk
    int64_t out;       // first row of the chunk's features in the output table
    uint64_t toa_min;  // smallest ToA of the chunk (sort fallback)
    int32_t tile0[4];  // first tile of each kind
};

struct SegSpec {
    int64_t start;
    int32_t count;
    uint64_t dt;
    int64_t out;
};

// Device pointers into one workspace, for n hits.
struct Work {
    int32_t n;
    // Non-null (single chunk only): the hit count lives in device memory,
    // written by an earlier kernel on the same stream; every kernel reads it
    // first and derives the tile counts from it, while n and the counts below
    // are capacity bounds that size the grids and the workspace.
    const int32_t* n_dev;
    uint32_t width, height;
    uint64_t dt;
    int32_t xcd_map;         // 1: contiguous tile ranges per XCD, 0: round-robin
    int32_t link_mode;       // 0: pixel index if the sensor's bitmap fits in LDS, else
                             // window scan; 1: pixel index (bitmap + CSR); 2: window scan
    int32_t n_seg;           // 1: one chunk, tile ranges computed arithmetically
    SegInfo* segs;           // n_seg > 1: chunk table
    int32_t* tile_seg[4];    // n_seg > 1: chunk of every tile, per kind
    // sort tiling
    int32_t sort_tile;   // T: hits per sort tile (power of two)
    int32_t sort_ipt;    // T / kSortThreads
    int32_t sort_m;      // neighbour tiles searched on each side
    int32_t n_sort_tiles;
    int32_t force_fallback;
    int32_t n_link_tiles;
    int32_t n_feat_tiles;
    int32_t n_scan_blocks;
    int32_t n_fb_blocks;
    int64_t edge_cap;        // kLinkHaloCap cross-tile edges per link tile
    int64_t carry_cap;       // kFeatHash carries per feature tile

    Status* status;
    TileInfo* tiles;
    uint32_t* tile_q;     // per sort tile, kTileQ keys: the last key of each of kTileQ equal parts (sorted, relative)
    uint32_t* ts_rel;     // tile-sorted ToA relative to the tile minimum
    uint2* ts_pay;        // tile-sorted payload: (local index | ToT << 16, x | y << 16)
    uint64_t* s_toa;
    uint32_t* s_xy;
    uint16_t* s_tot;
    int32_t* s_idx;
    int32_t* link_h0;     // per link tile: first halo position, or -1 if it overflows
    int32_t* gparent;
    int2* edges;
    int32_t* tile_nedge;     // cross-tile edges of every link tile
    int32_t* overflow_tiles;
    int32_t* deep_tiles;     // overflow tiles that go on to the link fallback
    int32_t* deep_ws;        // per link tile: its window's first sorted position if deep, else -1
    int32_t* run_off;        // per deep tile, in tile order: where its run of the windows' union starts (+ total)
    int32_t* run_base;       // per deep tile: the run's first sorted position
    int32_t* blk_run;        // per fallback radix block: the run holding its first element (+ last run)
    SlotRec* slots;
    SlotRec* carries;
    int32_t* tile_ncarry;    // carries of every feature tile
    uint32_t* blk_count;              // roots per block of kScanBlock indices
    uint32_t* blk_off;                // exclusive scan of blk_count
    unsigned long long* root_mask;    // one bit per input index: labels[i] == i
    uint16_t* root_wpre;              // per mask word: roots in the earlier words of its block
    uint64_t* fb_key[2];
    uint32_t* fb_val[2];
    uint32_t* fb_hist;
};

// Workspace planning (host).  With segs/n_seg > 1 the input is a batch of
// independent chunks; upload_segments then fills the chunk and tile tables.
size_t plan_workspace(int64_t n, uint32_t width, uint32_t height, uint32_t disorder, Work* w,
                      char* base, const SegSpec* segs = nullptr, int n_seg = 1);
int upload_segments(const Work& w, const SegSpec* segs, int n_seg, hipStream_t s, void* pinned_staging,
                    size_t staging_bytes);
size_t segment_table_bytes(const Work& w);

// Kernel launchers; each returns the hipError_t of its launch.
hipError_t launch_init(const Work& w, hipStream_t s);
hipError_t launch_tile_sort(const hc_hit* hits, const Work& w, hipStream_t s);
hipError_t launch_tile_merge(const Work& w, hipStream_t s);
hipError_t launch_link_halo(const Work& w, hipStream_t s);
hipError_t launch_sort_fallback(const hc_hit* hits, const Work& w, hipStream_t s);
hipError_t launch_link(const Work& w, hipStream_t s);
hipError_t launch_link_wide(const Work& w, hipStream_t s);
hipError_t launch_link_fallback(const Work& w, hipStream_t s);
hipError_t launch_union_edges(const Work& w, hipStream_t s);
hipError_t launch_flatten(const Work& w, int32_t* labels, hipStream_t s);
hipError_t launch_features(const Work& w, const int32_t* labels, hipStream_t s);
hipError_t launch_carries(const Work& w, hipStream_t s);
hipError_t launch_scan_blocks(const Work& w, int32_t* n_clusters, hipStream_t s);
hipError_t launch_compact(const Work& w, hc_features* features, hipStream_t s);
hipError_t launch_write_count(int32_t* n_clusters, int32_t value, hipStream_t s);

// The whole plain clustering sequence on one workspace (hc_api.cpp).
int enqueue_cluster(const hc_hit* hits, const Work& w, int32_t* labels, hc_features* features,
                    int32_t* n_clusters, hipStream_t s);
// Record an error for hc_last_error and return its code.
int set_error(int code, const std::string& msg);
// Sort tile for a displacement hint D: tiles of T hits ranked against
// m = ceil(2D / T) neighbour tiles per side.  4096-hit tiles with up to two
// neighbours measured faster than 8192-hit tiles with one (smaller LDS
// footprint, more work-groups per CU).
inline int sort_tile_for(int64_t D)
{
    if (2 * D <= 2048) return 2048;
    if (2 * D <= 8192) return 4096;
    return 8192;
}

// hc_opts.flags: at most one HC_FLAG_LINK_* value, optionally with
// HC_FLAG_GLOBAL_TIME (hc_cluster only); the Work.link_mode it selects.
inline bool link_flags_valid(uint32_t f)
{
    const uint32_t link = f & ~HC_FLAG_GLOBAL_TIME;
    return link == 0 || link == HC_FLAG_LINK_PIXEL_INDEX || link == HC_FLAG_LINK_WINDOW;
}
inline int32_t link_mode_of(const hc_opts* o)
{
    if (!o) return 0;
    const uint32_t link = o->flags & ~HC_FLAG_GLOBAL_TIME;
    return link == HC_FLAG_LINK_PIXEL_INDEX ? 1 : link == HC_FLAG_LINK_WINDOW ? 2 : 0;
}
inline bool global_time_of(const hc_opts* o) { return o && (o->flags & HC_FLAG_GLOBAL_TIME); }

// The Section 2 (iii)(b) clustering (hc_global.hip): its extra workspace
// (behind the plain path's), and the launch sequence.
struct GlbWork;
size_t plan_global(int64_t n, GlbWork* g, char* base);
int global_cluster(const hc_hit* hits, Work& w, char* extra, int32_t* labels, hc_features* features,
                   int32_t* n_clusters, hipStream_t s);
// Segments of the fallback's digit-counter scan (256 counters per block).
__host__ __device__ inline int32_t fb_scan_segments(int32_t nb)
{
    return (int32_t)(((int64_t)256 * nb + kFbScanSeg - 1) / kFbScanSeg);
}
// Cached workspace of (current device, stream s) for callers that pass none
// (grown on demand).  *hold keeps the buffer reserved for the caller until it
// has enqueued its work on s.
int cached_workspace(size_t need, hipStream_t s, void** out, std::unique_lock<std::mutex>* hold);
// Switch per-kernel event timing on or off; returns the previous state.
bool timing_set(bool on);
// Device memory of a stream (hc_stream_*): held now, and after a push of n
// hits (with the bytes alive only while its buffers grow in *transient).
size_t stream_device_bytes(const hc_stream* st);
size_t stream_bytes_after_push(const hc_stream* st, int64_t n, size_t* transient);
int64_t stream_open_hits(const hc_stream* st);
// Pushes enqueued so far, and pushes completed on the device and read back
// (retiring whatever has completed, without waiting); wait for the oldest
// push in flight.
uint64_t stream_pushes_enqueued(const hc_stream* st);
uint64_t stream_pushes_retired(hc_stream* st);
int stream_wait_one(hc_stream* st);
size_t stream_inflight(const hc_stream* st);
// A chunk of a completed push, as the server sees it: its tag, whether it was
// accepted, how many clusters the push closed (counted for the push's last
// chunk, 0 for the others), and whether it is the push's last chunk.
struct RetiredPush {
    uint64_t tag;
    int32_t verdict;
    int32_t n_closed;
    int32_t last;
};
// Chunks one push may carry.
constexpr int kMaxPushChunks = 16;
// Pushes in flight at most (depth); with log_retired every completed chunk
// push is recorded for stream_take_retired, which appends and clears them.
void stream_configure(hc_stream* st, int depth, bool log_retired);
size_t stream_take_retired(hc_stream* st, std::vector<RetiredPush>* out);
int set_device_error(hipError_t e, const char* what);
int persistent_grid();

// Kernel timing hooks (hc_api.cpp): bracket a launch with events when enabled.
struct TimedLaunch {
    TimedLaunch(const char* name, hipStream_t s);
    ~TimedLaunch();
    const char* name_;
    hipStream_t s_;
    int slot_;
};

}  // namespace hc

namespace hc {
// Occupancy bitmap of the link kernel's pixel index: one bit per sensor pixel
// plus a 16-bit prefix count per 64-bit word, in dynamic LDS (2.25 bits per
// pixel).  Sensors with more than kLinkMaxPixels pixels cannot use the index.
constexpr uint64_t kLinkMaxPixels = 448ull * 512ull;
}  // namespace hc
