// Hooking of accepted pairs, shared by the single-instance and batched
// post-processing (Algorithm 1: core points joined into components, other
// points offered their core neighbours).
#pragma once
#include "sng_internal.hpp"

namespace sng {

// uf_unite with a device-scope read of the root to be hooked just before the
// compare-and-swap. Where the threads of one launch hook many links between
// the same few large components, their cached walks keep returning a root
// that another XCD has already hooked; each such stale root costs a failing
// compare-and-swap, and those serialise on one address at the memory side.
// A fresh read of that address catches most of them for the price of a read.
__device__ __forceinline__ void uf_unite_verified(int32_t *P, int32_t a, int32_t b)
{
    int32_t ra = uf_find(P, a), rb = uf_find(P, b);
    while (ra != rb) {
        if (ra > rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        const int32_t now = ld_relaxed(P + rb);
        if (now == rb) {
            const int32_t old = atomicCAS(P + rb, rb, ra);
            if (old == rb)
                return;
            rb = old;
        } else {
            rb = now;
        }
        rb = uf_find(P, rb);
        ra = uf_find(P, ra);
    }
}

// One accepted pair (a, b): two core points join their components; a core
// and a non-core point offer the core index to the non-core point (atomic
// minimum, so the smallest core neighbour wins whatever the order). The
// union reads the root to be hooked at device scope first: a dense cluster's
// pairs keep meeting roots already hooked elsewhere (10k x 2 call 129 ->
// 110 us, 64-instance batch 23.6 -> 22.9 ms).
__device__ __forceinline__ void hook_pair(const Inst &I, uint32_t a, uint32_t b)
{
    const bool ca = I.core[a], cb = I.core[b];
    if (ca && cb)
        uf_unite_verified(I.labels, (int32_t)a, (int32_t)b);
    else if (ca)
        atomicMin(I.labels + b, (int32_t)a);
    else if (cb)
        atomicMin(I.labels + a, (int32_t)b);
}

// Block-local compaction of accept words: one round reads kHookRoundWords
// words (one per thread of a 256-thread block, starting at w0, none at or
// beyond hi) and lists their accepted slots in LDS, then every thread of
// the block regenerates list entries and hands each accepted pair (i, j) to
// f. A wavefront therefore handles about (accepted slots of the round) / 256
// pairs in sequence instead of one per (call, Philox word) position that any
// of its lanes accepted. w0 and hi must be the same for the whole block.
// Entry: word offset in the round * 32 + bit (call in the word * 4 + Philox
// word).
constexpr uint32_t kHookRoundWords = 256;

template <class F>
__device__ __forceinline__ void accepted_round(const Inst &I, uint64_t w0, uint64_t hi,
                                               uint16_t *list, uint32_t *nlist, F &&f)
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
        f(i, mod_exact(W.w[v & 3u], I.n, I.inv_n));
    }
    __syncthreads();  // the next round reuses the list and the count
}

// The hook of one round of accept words.
__device__ __forceinline__ void hook_round(const Inst &I, uint64_t w0, uint64_t hi,
                                           uint16_t *list, uint32_t *nlist)
{
    accepted_round(I, w0, hi, list, nlist, [&](uint32_t i, uint32_t j) { hook_pair(I, i, j); });
}

}  // namespace sng
