// hc_cluster_noalloc: hc_cluster for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The workspace is a fixed array in device memory,
// reserved when the library's code object is loaded on a device and held by
// that device until the process ends.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// the array's device address comes from hipGetSymbolAddress, taken once per
// device (with that device current) on the first call there, and only that
// address is ever handed to kernels.
#include <mutex>
#include <string>

#include "hc_device.h"

namespace {

constexpr size_t kScratchBytes = HC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device.
int scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hc::set_device_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return hc::set_error(HC_ERR_DEVICE, "device ordinal beyond the table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hc::set_device_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return hc::set_error(HC_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return HC_OK;
}

}  // namespace

using namespace hc;

extern "C" {

size_t hc_noalloc_scratch_bytes(void) { return kScratchBytes; }

int hc_cluster_noalloc(const hc_hit* hits, int32_t n, uint64_t dt, int32_t* labels, hc_features* features,
                       int32_t* n_clusters, const hc_opts* opts)
{
    if (n < 0) return set_error(HC_ERR_ARG, "n < 0");
    if (!n_clusters) return set_error(HC_ERR_ARG, "n_clusters is NULL");
    if (n > 0 && (!hits || !labels)) return set_error(HC_ERR_ARG, "hits or labels is NULL");
    const uint32_t W = opts && opts->width ? opts->width : 256;
    const uint32_t H = opts && opts->height ? opts->height : 256;
    if (W > 65535 || H > 65535) return set_error(HC_ERR_ARG, "sensor dimensions must be 1..65535");
    if (opts && !link_flags_valid(opts->flags)) return set_error(HC_ERR_ARG, "unknown flags");
    if (global_time_of(opts))
        return set_error(HC_ERR_ARG, "HC_FLAG_GLOBAL_TIME is not available without allocation");
    if (opts && opts->workspace)
        return set_error(HC_ERR_ARG, "hc_cluster_noalloc uses its own scratch; pass no workspace");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    void* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc != HC_OK) return rc;
    hipError_t e;
    if (n == 0) {
        if ((e = launch_write_count(n_clusters, 0, s)) != hipSuccess) return set_device_error(e, "write_count");
        return HC_OK;
    }
    const uint32_t D = opts ? opts->disorder_hint : 0;
    const size_t need = plan_workspace(n, W, H, D, nullptr, nullptr);
    if (need > kScratchBytes)
        return set_error(HC_ERR_WORKSPACE, "hc_cluster_noalloc: " + std::to_string(n) + " hits need " +
                                               std::to_string(need) + " bytes of scratch, the limit is " +
                                               std::to_string(kScratchBytes));
    Work w;
    plan_workspace(n, W, H, D, &w, (char*)ws);
    w.dt = dt;
    w.link_mode = link_mode_of(opts);
    // the path reads no workspace word it has not written in the same call
    // (its first kernel clears the status block), so whatever the previous
    // call left in the array does not matter
    return enqueue_cluster(hits, w, labels, features, n_clusters, s);
}

}  // extern "C"
