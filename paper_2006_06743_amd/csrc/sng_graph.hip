// Post-processing of SNG-DBSCAN (Algorithm 1, last three steps) on the
// device:
//   core init  core[i] = (int64)deg[i] >= MinPts; the label array becomes the
//              union-find parent for core points (parent = self) and the
//              "smallest core neighbour" slot for the others (empty);
//   hook       every accepted pair is regenerated from its slot bit (Philox
//              again, no distance work): a core-core pair joins the two
//              components, a core/non-core pair offers the core index to
//              the non-core point (atomic min);
//   finalize   core points take their root (the component's minimum index),
//              then non-core points take the label of their smallest core
//              neighbour, or -1.
// Roots are minimum indices whatever the order of the atomic operations, so
// the result is deterministic.
#include "sng_hook.hpp"

namespace sng {

__global__ void k_fill_u32(uint32_t *p, uint64_t count, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t count, unsigned long long v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Grid-stride launches: enough blocks to fill the chip, few enough that the
// per-block counter atomics stay cheap.
static unsigned grid_for(uint64_t items, unsigned block)
{
    uint64_t g = (items + block - 1) / block;
    if (g > 4096)
        g = 4096;
    return (unsigned)(g ? g : 1);
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t v, hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t count, unsigned long long v,
                           hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

__device__ __forceinline__ void count_add(unsigned long long *cnt, int slot, uint32_t mine)
{
    const int slots[1] = {slot};
    const uint32_t v[1] = {mine};
    block_count_add<1>(cnt, slots, v);
}

__global__ __launch_bounds__(256) void k_core_init(Inst I)
{
    uint32_t n_core = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const bool c = (int64_t)I.deg[i] >= (int64_t)I.min_pts;
        I.core[i] = c;
        I.labels[i] = c ? (int32_t)i : kNoCore;
        n_core += c;
    }
    count_add(I.cnt, kCntCore, n_core);
}

// Block-local compaction of the accept words (hook_round): a block lists
// the accepted slots of 256 words in LDS and its threads share them out, so
// the slots of a dense stretch of words are hooked side by side instead of
// one after another by the thread that holds their word. With the verified
// union (a fresh read of the root before each compare-and-swap) this beats one
// thread per accept word: 10k x 2 call 111 -> 78 us, 1e6 x 16 at sigma 0.25
// 13.66 -> 11.87 ms per call. Before that union, the same listing was slower
// (168 against 85 us on the 10k x 2 call): more hooks at once into the same
// few dense clusters cost more in failed compare-and-swaps than they hid.
__global__ __launch_bounds__(256) void k_hook_mask(Inst I)
{
    // Without a core point no pair joins or offers anything, and the accept
    // words (one bit per slot: 1.6 GB on the 5e6-point scene) need not be read.
    if (I.cnt && __hip_atomic_load(I.cnt + kCntCore, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) == 0ull)
        return;  // grid-uniform
    const uint64_t words = I.chunks * 8ull;
    __shared__ uint16_t list[kHookRoundWords * 32];
    __shared__ uint32_t nlist;
    for (uint64_t w0 = (uint64_t)blockIdx.x * kHookRoundWords; w0 < words;
         w0 += (uint64_t)gridDim.x * kHookRoundWords)  // block-uniform
        hook_round(I, w0, words, list, &nlist);
}

__global__ __launch_bounds__(256) void k_hook_edges(Inst I, const int32_t *edges, int64_t n_edges)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_edges;
         e += (int64_t)gridDim.x * blockDim.x)
        hook_pair(I, (uint32_t)edges[2 * e], (uint32_t)edges[2 * e + 1]);
}

__global__ __launch_bounds__(256) void k_edge_degrees(const int32_t *edges, int64_t n_edges,
                                                      uint32_t *deg)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_edges;
         e += (int64_t)gridDim.x * blockDim.x) {
        atomicAdd(deg + edges[2 * e], 1u);
        atomicAdd(deg + edges[2 * e + 1], 1u);
    }
}

hipError_t launch_core_init(const Inst &I, hipStream_t st)
{
    if (I.n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_core_init, dim3(grid_for(I.n, 256)), dim3(256), 0, st, I);
    return hipGetLastError();
}

hipError_t launch_hook_mask(const Inst &I, hipStream_t st, unsigned blocks)
{
    if (I.chunks == 0)
        return hipSuccess;
    const uint64_t words = I.chunks * 8ull;
    const uint64_t most = (words + kHookRoundWords - 1) / kHookRoundWords;  // one round per block
    unsigned g = grid_for(words, kHookRoundWords);
    if (blocks != 0)  // a tuned grid (the loop is grid-stride over rounds)
        g = (unsigned)(blocks < most ? blocks : most);
    hipLaunchKernelGGL(k_hook_mask, dim3(g), dim3(256), 0, st, I);
    return hipGetLastError();
}

hipError_t launch_hook_edges(const Inst &I, const int32_t *edges, int64_t n_edges, hipStream_t st)
{
    if (n_edges == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_hook_edges, dim3(grid_for((uint64_t)n_edges, 256)), dim3(256), 0, st, I,
                       edges, n_edges);
    return hipGetLastError();
}

hipError_t launch_edge_degrees(const int32_t *edges, int64_t n_edges, uint32_t *deg,
                               hipStream_t st)
{
    if (n_edges == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_edge_degrees, dim3(grid_for((uint64_t)n_edges, 256)), dim3(256), 0, st,
                       edges, n_edges, deg);
    return hipGetLastError();
}

// Both finalize steps in one launch: a core point takes the root of its
// component, a non-core point the root of its smallest core neighbour (or
// -1). Core entries are rewritten with their roots while other threads walk
// the forest; a rewrite only shortens a path to the same root, so every
// read-only walk still ends there. A non-core entry is read and written only
// by its own thread (core walks never pass through non-core points).
__global__ __launch_bounds__(256) void k_finalize(Inst I)
{
    uint32_t roots = 0, noise = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
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

hipError_t launch_finalize(const Inst &I, hipStream_t st)
{
    if (I.n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(I.n, 256)), dim3(256), 0, st, I);
    return hipGetLastError();
}

}  // namespace sng
