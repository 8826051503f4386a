// Batched SNG-DBSCAN: many independent instances (uneven sizes, one shared
// dimension) solved by one sequence of launches, each covering every
// instance. The sampled-distance pass walks a global sequence of 64-call
// chunks in which every instance starts on a chunk of its own; the per-point
// and per-accept-word passes give each block a range of exactly one
// instance (block prefix tables), so per-block counter reductions still
// belong to one instance. The sequence contains kernel launches only, so it
// can be recorded once into a HIP graph and replayed.
#include "sng_hook.hpp"

namespace sng {

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Instance k of the block, from an exclusive prefix of blocks per instance.
__device__ __forceinline__ int block_instance(const uint64_t *__restrict__ starts, int count,
                                              uint64_t b)
{
    int a = 0, z = count - 1;
    while (a < z) {
        const int mid = (a + z + 1) >> 1;
        if (starts[mid] <= b)
            a = mid;
        else
            z = mid - 1;
    }
    return a;
}

__device__ __forceinline__ void batch_count(unsigned long long *cnt, int slot, uint32_t mine)
{
    const int slots[1] = {slot};
    const uint32_t v[1] = {mine};
    block_count_add<1>(cnt, slots, v);
}

// Counters of every instance (first block of the instance) and degrees.
__global__ __launch_bounds__(256) void k_b_init(const Inst *__restrict__ T, const BatchGeom G)
{
    const int k = block_instance(G.pblk, G.count, blockIdx.x);
    const Inst &I = T[k];
    const uint64_t b = blockIdx.x - G.pblk[k];
    if (b == 0 && (threadIdx.x < kCntNum || (threadIdx.x > kCntNum && threadIdx.x < kFltEnd)))
        I.cnt[threadIdx.x] = (threadIdx.x == kCntSlots) ? (unsigned long long)I.n * I.m : 0ull;
    if (b == 0 && threadIdx.x == 0)
        reinterpret_cast<double *>(I.cnt)[kCntNum] = I.band;
    const uint64_t lo = b * kPointsPerBlock;
    const uint64_t hi = umin64(lo + kPointsPerBlock, I.n);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
        I.deg[i] = 0u;
}

__global__ __launch_bounds__(256) void k_b_core_init(const Inst *__restrict__ T, const BatchGeom G)
{
    const int k = block_instance(G.pblk, G.count, blockIdx.x);
    const Inst &I = T[k];
    const uint64_t lo = (blockIdx.x - G.pblk[k]) * kPointsPerBlock;
    const uint64_t hi = umin64(lo + kPointsPerBlock, I.n);
    uint32_t n_core = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const bool c = (int64_t)I.deg[i] >= (int64_t)I.min_pts;
        I.core[i] = c;
        I.labels[i] = c ? (int32_t)i : kNoCore;
        n_core += c;
    }
    batch_count(I.cnt, kCntCore, n_core);
}

// Hook of the accept words of one instance range, a round of
// kHookRoundWords words at a time with block-local compaction.
// Grid: total_wblocks rounded up to whole eighths; each XCD hooks a
// contiguous eighth of the word blocks (xcd_block), so an instance's labels
// and core flags stay in one L2.
__global__ __launch_bounds__(256) void k_b_hook(const Inst *__restrict__ T, const BatchGeom G)
{
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= G.total_wblocks)
        return;  // block-uniform
    const int k = block_instance(G.wblk, G.count, blk);
    const Inst &I = T[k];
    const uint64_t words = I.chunks * 8ull;
    const uint64_t lo = (blk - G.wblk[k]) * kWordsPerBlock;
    const uint64_t hi = umin64(lo + kWordsPerBlock, words);
    __shared__ uint16_t list[kHookRoundWords * 32];
    __shared__ uint32_t nlist;
    for (uint64_t w0 = lo; w0 < hi; w0 += kHookRoundWords)  // block-uniform
        hook_round(I, w0, hi, list, &nlist);
}

// Both finalize steps of the instance's point range in one launch, as in the
// single-instance finalize: core points take their root, non-core points the
// root of their smallest core neighbour (read-only walks, which the
// concurrent root rewrites only shorten), or -1.
__global__ __launch_bounds__(256) void k_b_finalize(const Inst *__restrict__ T, const BatchGeom G)
{
    const int k = block_instance(G.pblk, G.count, blockIdx.x);
    const Inst &I = T[k];
    const uint64_t lo = (blockIdx.x - G.pblk[k]) * kPointsPerBlock;
    const uint64_t hi = umin64(lo + kPointsPerBlock, I.n);
    uint32_t roots = 0, noise = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (I.core[i]) {
            const int32_t r = uf_root(I.labels, (int32_t)i);
            st_relaxed(I.labels + i, r);
            roots += (r == (int32_t)i);
        } else {
            const int32_t b = I.labels[i];
            const int32_t l = (b == kNoCore) ? -1 : uf_root(I.labels, b);
            I.labels[i] = l;
            noise += (l == -1);
        }
    }
    const int slots[2] = {kCntClusters, kCntNoise};
    const uint32_t v[2] = {roots, noise};
    block_count_add<2>(I.cnt, slots, v);
}

hipError_t launch_batch(const Inst *T, const BatchGeom &G, int d, bool vec_ok,
                        const PassAShape &sh, hipStream_t st)
{
    hipError_t e;
    if (G.count == 0)
        return hipSuccess;
    const unsigned pb = (unsigned)G.total_pblocks, wb = (unsigned)G.total_wblocks;
    hipLaunchKernelGGL(k_b_init, dim3(pb), dim3(256), 0, st, T, G);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (G.total_chunks > 0) {
        e = launch_pass_a_batch(T, G.count, G.chunk_starts, G.total_chunks, d, vec_ok, sh, st);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_b_core_init, dim3(pb), dim3(256), 0, st, T, G);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (wb > 0) {
        hipLaunchKernelGGL(k_b_hook, dim3((wb + 7) / 8 * 8), dim3(256), 0, st, T, G);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_b_finalize, dim3(pb), dim3(256), 0, st, T, G);
    return hipGetLastError();
}

}  // namespace sng
