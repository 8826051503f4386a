// Simple-graph degrees: the sampled graph of Algorithm 1 read as a simple
// graph, so a point's degree is its number of distinct accepted neighbours,
// a pair sampled several times, by either endpoint, counting once.
//
// After the sampled-distance pass every accepted slot is regenerated from
// its accept bit (Philox again, no distance work) and its pair {min, max}
// is inserted into an open-addressing hash table of 64-bit keys with linear
// probing; only the insertion that finds its key absent adds one to both
// degrees. The table has 2^b entries, b chosen on the device from the
// accepted count so that at most half of them fill: probing always meets an
// empty entry, and clearing costs time in proportion to the accepted pairs,
// not to the workspace's largest table.
#include "sng_internal.hpp"
#include "sng_hook.hpp"

namespace sng {

namespace {

constexpr unsigned long long kEmpty = ~0ull;  // no key: min < max < 2^31

__global__ void k_simple_size(const unsigned long long *cnt, uint32_t max_log2,
                              uint32_t *log2_out)
{
    if (threadIdx.x != 0)
        return;
    const unsigned long long want = 2ull * cnt[kCntAccepted];
    uint32_t b = max_log2 < 6 ? max_log2 : 6;
    while (b < max_log2 && (1ull << b) < want)
        ++b;
    *log2_out = b;
}

__global__ __launch_bounds__(256) void k_simple_clear(unsigned long long *table,
                                                      const uint32_t *log2p)
{
    const uint64_t cap = 1ull << *log2p;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cap;
         e += (uint64_t)gridDim.x * blockDim.x)
        table[e] = kEmpty;
}

__device__ __forceinline__ void simple_insert(uint32_t *deg, unsigned long long *table,
                                              uint32_t b, uint32_t i, uint32_t j)
{
    const uint32_t lo = i < j ? i : j, hi = i < j ? j : i;
    const unsigned long long key = ((unsigned long long)lo << 32) | hi;
    const uint64_t mask = (1ull << b) - 1;
    // Fibonacci hashing: the top b bits of key * 2^64 / golden ratio
    uint64_t h = (b == 0) ? 0 : (uint64_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - b));
    for (uint64_t probe = 0; probe <= mask; ++probe) {  // at most half full: ends early
        const unsigned long long old = atomicCAS(table + h, kEmpty, key);
        if (old == kEmpty) {
            atomicAdd(deg + lo, 1u);
            atomicAdd(deg + hi, 1u);
            return;
        }
        if (old == key)
            return;
        h = (h + 1) & mask;
    }
}

// Accepted slots listed per block and shared out, as in the hook (one thread
// per accept word: 1e6 x 16 at sigma 0.25 15.0 ms per call, 10k x 2 136 us;
// listed: 14.6 ms and 108 us).
__global__ __launch_bounds__(256) void k_simple_insert(Inst I, unsigned long long *table,
                                                       const uint32_t *log2p)
{
    const uint32_t b = *log2p;
    const uint64_t words = I.chunks * 8ull;
    __shared__ uint16_t list[kHookRoundWords * 32];
    __shared__ uint32_t nlist;
    for (uint64_t w0 = (uint64_t)blockIdx.x * kHookRoundWords; w0 < words;
         w0 += (uint64_t)gridDim.x * kHookRoundWords)  // block-uniform
        accepted_round(I, w0, words, list, &nlist,
                       [&](uint32_t i, uint32_t j) { simple_insert(I.deg, table, b, i, j); });
}

unsigned grid_for(uint64_t items)
{
    uint64_t g = (items + 255) / 256;
    g = g > 4096 ? 4096 : (g ? g : 1);
    return (unsigned)g;
}

}  // namespace

uint32_t simple_table_log2(int64_t n, int64_t m)
{
    const uint64_t want = 2ull * (uint64_t)n * (uint64_t)m;
    uint32_t b = 6;
    while (b < 63 && (1ull << b) < want)
        ++b;
    return b;
}

hipError_t launch_simple_degrees(const Inst &I, unsigned long long *table, uint32_t max_log2,
                                 uint32_t *log2_word, hipStream_t st)
{
    hipError_t e = launch_fill_u32(I.deg, I.n, 0u, st);
    if (e != hipSuccess || I.n == 0 || I.m == 0)
        return e;
    hipLaunchKernelGGL(k_simple_size, dim3(1), dim3(64), 0, st, I.cnt, max_log2, log2_word);
    // the cleared size is read on the device; 4096 blocks cover any table
    hipLaunchKernelGGL(k_simple_clear, dim3(4096), dim3(256), 0, st, table, log2_word);
    hipLaunchKernelGGL(k_simple_insert, dim3(grid_for(I.chunks * 8ull)), dim3(256), 0, st, I,
                       table, log2_word);
    return hipGetLastError();
}

}  // namespace sng
