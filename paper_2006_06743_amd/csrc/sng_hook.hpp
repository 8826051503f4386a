// Hooking of accepted pairs, shared by the single-instance and batched
// post-processing (Algorithm 1: core points joined into components, other
// points offered their core neighbours).
#pragma once
#include "sng_internal.hpp"

namespace sng {

// One accepted pair (a, b): two core points join their components; a core
// and a non-core point offer the core index to the non-core point (atomic
// minimum, so the smallest core neighbour wins whatever the order).
__device__ __forceinline__ void hook_pair(const Inst &I, uint32_t a, uint32_t b)
{
    const bool ca = I.core[a], cb = I.core[b];
    if (ca && cb)
        uf_unite(I.labels, (int32_t)a, (int32_t)b);
    else if (ca)
        atomicMin(I.labels + b, (int32_t)a);
    else if (cb)
        atomicMin(I.labels + a, (int32_t)b);
}

// Block-local compaction of accept words: one round reads kHookRoundWords
// words (one per thread of a 256-thread block, starting at w0, none at or
// beyond hi) and lists their accepted slots in LDS, then every thread of
// the block regenerates and hooks list entries. A wavefront therefore runs
// about (accepted slots of the round) / 256 hooks in sequence instead of one
// per (call, Philox word) position that any of its lanes accepted. w0 and hi
// must be the same for the whole block. Entry: word offset in the round * 32
// + bit (call in the word * 4 + Philox word).
constexpr uint32_t kHookRoundWords = 256;

__device__ __forceinline__ void hook_round(const Inst &I, uint64_t w0, uint64_t hi,
                                           uint16_t *list, uint32_t *nlist)
{
    if (threadIdx.x == 0)
        *nlist = 0;
    const uint64_t w = w0 + threadIdx.x;
    const uint32_t bits = (w < hi) ? I.mask[I.chunk0 * 8ull + w] : 0u;
    if (!__syncthreads_or(bits != 0u))
        return;  // no accepted slot in this round (the list is not read)
    uint32_t pos = list_reserve((uint32_t)__builtin_popcount(bits), nlist);
    for (uint32_t b = bits; b; b &= b - 1)
        list[pos++] = (uint16_t)(threadIdx.x * 32u + (uint32_t)__builtin_ctz(b));
    __syncthreads();
    const uint32_t cnt = *nlist;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const uint32_t v = list[e];
        const uint64_t call = (w0 + (v >> 5)) * 8ull + ((v & 31u) >> 2);
        const uint32_t i = (uint32_t)div_exact64(call, I.C, I.inv_C);
        const uint32_t c = (uint32_t)(call - (uint64_t)i * I.C);
        const Words4 W = philox10(c, i, I.key0, I.key1);
        hook_pair(I, i, mod_exact(W.w[v & 3u], I.n, I.inv_n));
    }
    __syncthreads();  // the next round reuses the list and the count
}

}  // namespace sng
