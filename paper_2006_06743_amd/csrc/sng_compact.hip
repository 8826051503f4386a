// Compact cluster ids. The clustering calls label every clustered point with
// the smallest core index of its component (its root r, labels[r] == r) and
// noise with -1; the method defines clusters only up to a renaming
// (Section 4.1, Theorem 1). This renames the roots 0..k-1 in increasing
// order without any workspace: the output array itself holds the per-tile
// root counts and their prefix until the final values overwrite them.
//
//   count   tile t (kTile labels) counts its roots into out[t*kTile]
//   scan    one workgroup turns those counts into exclusive tile offsets
//   roots   tile t reads its offset, ranks its roots in index order and
//           writes out[r] for every root r of the tile
//   gather  every non-root i takes out[labels[i]] (a root's slot, final
//           since the previous kernel) or -1
#include "sng_internal.hpp"

namespace sng {

namespace {

constexpr uint32_t kTile = 4096;         // labels per tile
constexpr uint32_t kTileThreads = 256;   // 16 consecutive labels per thread
constexpr uint32_t kPerThread = kTile / kTileThreads;
constexpr uint32_t kScanThreads = 1024;

__device__ __forceinline__ bool is_root(const int32_t *labels, uint32_t i)
{
    return labels[i] == (int32_t)i;
}

// Exclusive prefix of v over the workgroup (blockDim.x threads, at most
// 1024), and the workgroup total in *total.
__device__ uint32_t block_exclusive(uint32_t v, uint32_t *lds, uint32_t *total)
{
    const uint32_t t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (uint32_t s = 1; s < blockDim.x; s <<= 1) {
        const uint32_t add = t >= s ? lds[t - s] : 0u;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const uint32_t incl = lds[t];
    *total = lds[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kTileThreads) void k_cmp_count(const int32_t *__restrict__ labels,
                                                            uint32_t n, int32_t *out)
{
    __shared__ uint32_t lds[kTileThreads];
    const uint32_t base = blockIdx.x * kTile;
    const uint32_t lo = base + threadIdx.x * kPerThread;
    uint32_t c = 0;
    for (uint32_t k = 0; k < kPerThread; ++k)
        c += (lo + k < n) && is_root(labels, lo + k);
    uint32_t total;
    block_exclusive(c, lds, &total);
    if (threadIdx.x == 0)
        out[base] = (int32_t)total;
}

__global__ __launch_bounds__(kScanThreads) void k_cmp_scan(int32_t *out, uint32_t tiles,
                                                           int32_t *n_clusters)
{
    __shared__ uint32_t lds[kScanThreads];
    const uint32_t per = (tiles + kScanThreads - 1) / kScanThreads;
    const uint32_t t0 = threadIdx.x * per;
    const uint32_t t1 = min(t0 + per, tiles);
    uint32_t c = 0;
    for (uint32_t t = t0; t < t1; ++t)
        c += (uint32_t)out[(uint64_t)t * kTile];
    uint32_t total;
    uint32_t run = block_exclusive(c, lds, &total);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t v = (uint32_t)out[(uint64_t)t * kTile];
        out[(uint64_t)t * kTile] = (int32_t)run;
        run += v;
    }
    if (threadIdx.x == 0 && n_clusters)
        *n_clusters = (int32_t)total;
}

__global__ __launch_bounds__(kTileThreads) void k_cmp_roots(const int32_t *__restrict__ labels,
                                                            uint32_t n, int32_t *out)
{
    __shared__ uint32_t lds[kTileThreads];
    __shared__ uint32_t offset;
    const uint32_t base = blockIdx.x * kTile;
    if (threadIdx.x == 0)
        offset = (uint32_t)out[base];
    // block_exclusive's barriers order this read and write of the offset
    // before every use of it and before any write to out below
    const uint32_t lo = base + threadIdx.x * kPerThread;
    uint32_t flags = 0;
    for (uint32_t k = 0; k < kPerThread; ++k)
        flags |= (uint32_t)((lo + k < n) && is_root(labels, lo + k)) << k;
    uint32_t total;
    uint32_t rank = block_exclusive((uint32_t)__builtin_popcount(flags), lds, &total);
    rank += offset;
    for (uint32_t k = 0; k < kPerThread; ++k) {
        if (flags >> k & 1u)
            out[lo + k] = (int32_t)rank++;
    }
}

__global__ __launch_bounds__(256) void k_cmp_gather(const int32_t *__restrict__ labels, uint32_t n,
                                                    int32_t *out)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t L = labels[i];
        if (L == (int32_t)i)
            continue;  // a root: written by k_cmp_roots
        int32_t v = -1;
        if (L >= 0 && (uint32_t)L < n && is_root(labels, (uint32_t)L))
            v = out[L];
        out[i] = v;
    }
}

}  // namespace

hipError_t launch_compact(const int32_t *labels, uint32_t n, int32_t *out, int32_t *n_clusters,
                          hipStream_t st)
{
    if (n == 0) {
        if (n_clusters)
            return launch_fill_u32((uint32_t *)n_clusters, 1, 0u, st);
        return hipSuccess;
    }
    const uint32_t tiles = (uint32_t)(((uint64_t)n + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_cmp_count, dim3(tiles), dim3(kTileThreads), 0, st, labels, n, out);
    hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(kScanThreads), 0, st, out, tiles, n_clusters);
    hipLaunchKernelGGL(k_cmp_roots, dim3(tiles), dim3(kTileThreads), 0, st, labels, n, out);
    const uint64_t want = ((uint64_t)n + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_cmp_gather, dim3(blocks), dim3(256), 0, st, labels, n, out);
    return hipGetLastError();
}

}  // namespace sng
