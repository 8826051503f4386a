// Allocation-free form of sng_dbscan, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid allocation). The workspace is a file-scope device array of fixed
// size, `scratch`, one copy per GPU, held until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: in host
// code that name is only a stand-in for the device symbol. The device address
// of each GPU's copy comes from hipGetSymbolAddress, called once per device
// with that device current, and is the only handle used afterwards.
#include <mutex>

#include "../../include/sng.h"
#include <hip/hip_runtime.h>

namespace {

constexpr size_t kScratchBytes = SNG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];  // device address of each GPU's copy, once resolved

// Device address of the current GPU's copy of `scratch`, resolved on the
// first call on that device; nullptr if HIP reports an error.
void *scratch_address()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" int sng_dbscan_noalloc(const float *X, int64_t n, int32_t d, int64_t ld, double s,
                                  double eps, int32_t min_pts, uint64_t seed, int32_t *labels,
                                  uint32_t *degrees, const sng_config *cfg, void *stream)
{
    if (cfg && cfg->reuse_sample)
        return SNG_EINVAL;  // the array is shared by every call on the GPU
    int64_t m = 0;
    int rc = sng_samples_per_point(s, n, &m);
    if (rc != SNG_OK)
        return rc;
    // the workspace sng_dbscan needs for direct gathers (the smallest form)
    const int32_t flags =
        SNG_FP32 | SNG_WS_DIRECT | ((cfg && cfg->simple_graph) ? SNG_WS_SIMPLE_GRAPH : 0);
    size_t need = 0;
    if ((rc = sng_workspace_size(n, d, m, flags, &need)) != SNG_OK)
        return rc;
    if (need > kScratchBytes)
        return SNG_ERANGE;
    void *ws = scratch_address();
    if (!ws)
        return SNG_EHIP;
    // sng_dbscan validates the rest, ignores the workspace's contents on entry
    // and clears what it uses with kernels (no memset, no allocation); the
    // partner-block schedule runs only if its records fit in the array too
    return sng_dbscan(X, n, d, ld, s, eps, min_pts, seed, labels, degrees, ws, kScratchBytes, cfg,
                      stream);
}
