// Batched SNG-DBSCAN: many independent instances (uneven sizes, one shared
// dimension) solved by one sequence of launches, each covering every
// instance. The sampled-distance pass walks a global sequence of 64-call
// chunks in which every instance starts on a chunk of its own; the per-point
// and per-accept-word passes give each block a range of exactly one
// instance (block prefix tables), so per-block counter reductions still
// belong to one instance. The sequence contains kernel launches only, so it
// can be recorded once into a HIP graph and replayed.
#include "sng_internal.hpp"

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
    if (b == 0 && threadIdx.x < kCntNum)
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

__device__ __forceinline__ void b_hook_pair(const Inst &I, uint32_t a, uint32_t b)
{
    const bool ca = I.core[a], cb = I.core[b];
    if (ca && cb)
        uf_unite(I.labels, (int32_t)a, (int32_t)b);
    else if (ca)
        atomicMin(I.labels + b, (int32_t)a);
    else if (cb)
        atomicMin(I.labels + a, (int32_t)b);
}

// Hook of the accept words of one instance range, with block-local
// compaction: a round scans 256 words (one per thread) and lists the
// accepted slots in LDS, then all threads regenerate and hook them. Entry:
// word offset in the round * 32 + bit (call in the word * 4 + Philox word).
constexpr uint32_t kBHookWords = 256;

// Grid: total_wblocks rounded up to whole eighths; each XCD hooks a
// contiguous eighth of the word blocks (xcd_block), so an instance's labels
// and core flags stay in one L2.
__global__ __launch_bounds__(256) void k_b_hook(const Inst *__restrict__ T, const BatchGeom G)
{
    __shared__ uint16_t list[kBHookWords * 32];
    __shared__ uint32_t nlist;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= G.total_wblocks)
        return;  // block-uniform
    const int k = block_instance(G.wblk, G.count, blk);
    const Inst &I = T[k];
    const uint64_t words = I.chunks * 8ull;
    const uint64_t lo = (blk - G.wblk[k]) * kWordsPerBlock;
    const uint64_t hi = umin64(lo + kWordsPerBlock, words);
    for (uint64_t w0 = lo; w0 < hi; w0 += kBHookWords) {  // block-uniform
        if (threadIdx.x == 0)
            nlist = 0;
        const uint64_t w = w0 + threadIdx.x;
        const uint32_t bits = (w < hi) ? I.mask[I.chunk0 * 8ull + w] : 0u;
        if (!__syncthreads_or(bits != 0u))
            continue;  // no accepted slot in this round (the list is not read)
        uint32_t pos = list_reserve((uint32_t)__builtin_popcount(bits), &nlist);
        for (uint32_t b = bits; b; b &= b - 1)
            list[pos++] = (uint16_t)(threadIdx.x * 32u + (uint32_t)__builtin_ctz(b));
        __syncthreads();
        const uint32_t cnt = nlist;
        for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            const uint32_t v = list[e];
            const uint64_t call = (w0 + (v >> 5)) * 8ull + ((v & 31u) >> 2);
            const uint32_t i = (uint32_t)div_exact64(call, I.C, I.inv_C);
            const uint32_t c = (uint32_t)(call - (uint64_t)i * I.C);
            const Words4 W = philox10(c, i, I.key0, I.key1);
            b_hook_pair(I, i, mod_exact(W.w[v & 3u], I.n, I.inv_n));
        }
        __syncthreads();  // the next round reuses the list
    }
}

__global__ __launch_bounds__(256) void k_b_compress(const Inst *__restrict__ T, const BatchGeom G)
{
    const int k = block_instance(G.pblk, G.count, blockIdx.x);
    const Inst &I = T[k];
    const uint64_t lo = (blockIdx.x - G.pblk[k]) * kPointsPerBlock;
    const uint64_t hi = umin64(lo + kPointsPerBlock, I.n);
    uint32_t roots = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (I.core[i]) {
            const int32_t r = uf_root(I.labels, (int32_t)i);
            st_relaxed(I.labels + i, r);
            roots += (r == (int32_t)i);
        }
    }
    batch_count(I.cnt, kCntClusters, roots);
}

__global__ __launch_bounds__(256) void k_b_borders(const Inst *__restrict__ T, const BatchGeom G)
{
    const int k = block_instance(G.pblk, G.count, blockIdx.x);
    const Inst &I = T[k];
    const uint64_t lo = (blockIdx.x - G.pblk[k]) * kPointsPerBlock;
    const uint64_t hi = umin64(lo + kPointsPerBlock, I.n);
    uint32_t noise = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (!I.core[i]) {
            const int32_t b = I.labels[i];
            const int32_t l = (b == kNoCore) ? -1 : I.labels[b];
            I.labels[i] = l;
            noise += (l == -1);
        }
    }
    batch_count(I.cnt, kCntNoise, noise);
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
    hipLaunchKernelGGL(k_b_compress, dim3(pb), dim3(256), 0, st, T, G);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_b_borders, dim3(pb), dim3(256), 0, st, T, G);
    return hipGetLastError();
}

}  // namespace sng
