// Sampled-distance pass scheduled for L2 reuse.
//
// Sample slots are uniform over all partners, so a direct gather reads one
// random row of X per slot; rows narrower than an L2 line (128 B) waste the
// rest of the line, and none is reused. This schedule first sorts the slots
// by partner block and then evaluates them block by block:
//
//   generate  one workgroup per range of kRangeCalls Philox calls. Each
//             non-self slot becomes a 4-byte record (call offset in the
//             range, word, partner offset in its partner block of 2^bshift
//             rows, about half a MB of X). The workgroup counting-sorts its
//             records by partner block in LDS and copies them out in order,
//             so its region of the record array is written with contiguous
//             stores, one segment per partner block;
//   evaluate  partner blocks are dealt to the eight XCDs (block J to XCD
//             J mod 8; workgroup b runs on XCD b mod 8). The wavefronts of
//             one XCD take the segments of its blocks in block-major order
//             from a shared counter, so they all work on one or two partner
//             blocks at a time and those rows stay in that XCD's L2. Source
//             rows are read in generator order, which streams through X.
//
// Decisions are the plain path's (binary32 band, binary64 recheck), so
// degrees, accept bits and labels are identical to the direct schedule.
#include <string.h>

#include "sng_bucket_eval.hpp"

namespace sng {


// ---------------------------------------------------------------------------
// Generate. LDS: the record stage of the range, then counts and offsets per
// partner block.
// ---------------------------------------------------------------------------
constexpr uint32_t kGenThreads = 1024;
constexpr uint32_t kCallsPerThread = (uint32_t)kRangeCalls / kGenThreads;
constexpr uint32_t kRangeSlots = 4 * (uint32_t)kRangeCalls;
static_assert(kCallsPerThread * kGenThreads == kRangeCalls, "range split");
static_assert(kRangeCalls <= (1u << (32 - kRecOffShift)), "call offset field");
static_assert(kMaxPartnerBlocks <= kGenThreads, "one count per thread in the prefix");

// Exclusive prefix of v over a workgroup of kGenThreads threads; *total gets
// the sum. wsum: kGenThreads / kWave words of LDS.
__device__ __forceinline__ uint32_t gen_exclusive(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const uint32_t u = __shfl_up(x, s);
        if (lane >= s)
            x += u;
    }
    if (lane == kWave - 1)
        wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < (int)(kGenThreads / kWave); ++k) {
        const uint32_t s = wsum[k];
        before += (k < w) ? s : 0u;
        all += s;
    }
    *total = all;
    return before + x - v;
}

// kMod: 0 the binary64 remainder, 1 the binary32 one, 2 the binary32 one
// with a 24-bit multiply (n < 2^24).
template <int kMod>
__global__ __launch_bounds__(kGenThreads) void k_bkt_generate(Inst I, BucketGeom B)
{
    extern __shared__ uint32_t lds_u32[];
    __shared__ uint32_t wsum[kGenThreads / kWave];
    // counts and offsets per partner block first, so that their LDS
    // addresses are small constants plus the block index
    uint32_t *cnt = lds_u32;               // [NJ]
    uint32_t *pre = cnt + B.NJ;            // [NJ]
    uint32_t *stage = pre + B.NJ;          // [kRangeSlots]
    const uint32_t tid = threadIdx.x;
    const uint64_t r = blockIdx.x;
    const uint64_t call_lo = r * kRangeCalls;
    const uint64_t call_hi = min(call_lo + kRangeCalls, I.calls);
    const uint32_t i0 = (uint32_t)(call_lo / I.C);
    const uint32_t c0 = (uint32_t)(call_lo - (uint64_t)i0 * I.C);
    for (uint32_t k = tid; k < B.NJ; k += kGenThreads)
        cnt[k] = 0;
    if (tid == 0) {
        B.start[2 * r + 0] = i0;  // source and call of the range's first call
        B.start[2 * r + 1] = c0;
    }
    __syncthreads();
    // this thread's calls are c0 + tid + k * kGenThreads of the range: the
    // first split into (source, call within the point) by one division, the
    // next ones advanced by kGenThreads = step_q * C + step_r calls
    uint32_t cc = c0 + tid, ii = i0;
    if (cc >= I.C) {
        const uint32_t q = div_exact(cc, I.C, I.inv_C);
        ii += q;
        cc -= q * I.C;
    }
    const uint32_t step_q = kGenThreads / I.C;
    const uint32_t step_r = kGenThreads - step_q * I.C;
    const uint32_t pmask = (1u << B.bshift) - 1u;
    // key: partner block << 16 | rank of the record within its block
    uint32_t key[4 * kCallsPerThread], rec[4 * kCallsPerThread];
    uint32_t self = 0;
#pragma unroll
    for (uint32_t c = 0; c < kCallsPerThread; ++c) {
        const uint32_t off = c * kGenThreads + tid;
        const bool live = call_lo + off < call_hi;
        const uint32_t nvalid = live ? min(4u, I.m - 4u * cc) : 0u;
        const Words4 W = philox10(cc, ii, I.key0, I.key1);
        // the record's fields other than the partner and its word
        const uint32_t hi_bits = B.lds ? (((ii - i0) << B.tc_bits) | cc) << (B.bshift + 2)
                                       : (off << kRecOffShift);
        const uint32_t w_shift = B.lds ? B.bshift : 16u;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint32_t kk = ~0u, rr = 0;
            if ((uint32_t)w < nvalid) {
                const uint32_t j = kMod == 2   ? mod_f32_n24(W.w[w], I.n, I.inv_nf)
                                   : kMod == 1 ? mod_f32(W.w[w], I.n, I.inv_nf)
                                               : mod_exact(W.w[w], I.n, I.inv_n);
                if (j == ii) {
                    ++self;
                } else {
                    const uint32_t J = j >> B.bshift;
                    kk = (J << 16) | atomicAdd(cnt + J, 1u);
                    rr = hi_bits | ((uint32_t)w << w_shift) | (j & pmask);
                }
            }
            key[4 * c + w] = kk;
            rec[4 * c + w] = rr;
        }
        cc += step_r;
        ii += step_q;
        if (cc >= I.C) {
            cc -= I.C;
            ++ii;
        }
    }
    __syncthreads();
    const uint32_t v = tid < B.NJ ? cnt[tid] : 0u;
    uint32_t total;
    const uint32_t ex = gen_exclusive(v, wsum, &total);
    if (tid < B.NJ) {
        pre[tid] = ex;
        B.seg[(r * B.NJ + tid) * 2 + 0] = ex;
        B.seg[(r * B.NJ + tid) * 2 + 1] = v;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < 4 * kCallsPerThread; ++k) {
        if (key[k] != ~0u)
            stage[pre[key[k] >> 16] + (key[k] & 0xFFFFu)] = rec[k];
    }
    __syncthreads();
    uint32_t *dst = B.rec + r * B.region;
    // stage starts 2*NJ words into LDS: copy out in 16-byte pieces when that
    // keeps both sides aligned, else word by word
    if ((B.NJ & 1u) == 0) {
        for (uint32_t k = 4 * tid; k < total; k += 4 * kGenThreads) {
            if (k + 4 <= total) {
                *reinterpret_cast<uint4 *>(dst + k) = *reinterpret_cast<const uint4 *>(stage + k);
            } else {
                for (uint32_t e = k; e < total; ++e)
                    dst[e] = stage[e];
            }
        }
    } else {
        for (uint32_t k = tid; k < total; k += kGenThreads)
            dst[k] = stage[k];
    }
    const int slots[1] = {1};
    const uint32_t sv[1] = {self};
    block_count_add<1>(B.hdr, slots, sv);
}

// Before generate: no valid sample, no self pairs counted yet.
__global__ void k_bkt_prepare(BucketGeom B, int clear_sample)
{
    const int t = threadIdx.x;
    if (t < kXcds)
        B.queue[t] = 0ull;
    if (clear_sample && t < 2)
        B.hdr[t] = 0ull;
}

// After generate: the records now hold the sample of B.tag.
__global__ void k_bkt_seal(BucketGeom B)
{
    if (threadIdx.x == 0)
        B.hdr[0] = B.tag;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
bool bucket_geometry(int64_t n, int d, int64_t m, bool force, BucketGeom *g)
{
    BucketGeom b;
    memset(&b, 0, sizeof(b));
    if (n < 1 || m < 1 || d > 32)
        return false;
    // chosen automatically only for rows narrower than an L2 line, and only
    // when X does not fit one XCD's L2
    if (!force && (d * 4 >= 128 || (uint64_t)n * (uint64_t)d * 4 <= ((uint64_t)8 << 20)))
        return false;
    // partner block: rows of at most kLdsMaxD floats take the largest power
    // of two of rows that fits kLdsBlockBytes (the evaluate kernel then holds
    // a whole block in LDS), unless that makes more than kMaxPartnerBlocks
    // blocks; otherwise at most 2^16 rows and about half a MB of rows, which
    // stay in one XCD's L2
    auto blocks_of = [&](int bs) { return (uint64_t)((n + ((int64_t)1 << bs) - 1) >> bs); };
    const uint64_t C = (uint64_t)((m + 3) / 4);
    int bs = 16;
    if (d <= kLdsMaxD) {
        while (bs > 6 && ((uint64_t)1 << bs) * (uint64_t)d * 4 > kLdsBlockBytes)
            --bs;
        // the LDS record fields: the call within the point (< C) and the
        // source's offset within its range (at most (C - 1 + kRangeCalls - 1) / C)
        uint32_t tc = 0, so = 0;
        while (((uint64_t)1 << tc) < C)
            ++tc;
        const uint64_t max_off = (C - 1 + kRangeCalls - 1) / C;
        while (((uint64_t)1 << so) <= max_off)
            ++so;
        b.tc_bits = tc;
        b.lds = (blocks_of(bs) <= kMaxPartnerBlocks && (uint32_t)bs + 2 + tc + so <= 32) ? 1u : 0u;
    }
    if (!b.lds) {
        bs = 16;
        while (bs > 6 && ((uint64_t)1 << bs) * (uint64_t)d * 4 > (512u << 10))
            --bs;
    }
    b.bshift = (uint32_t)bs;
    if (blocks_of(bs) > kMaxPartnerBlocks)
        return false;
    b.NJ = (uint32_t)blocks_of(bs);
    const uint64_t calls = (uint64_t)n * C;
    b.ranges = (calls + kRangeCalls - 1) / kRangeCalls;
    b.region = kRangeSlots;
    uint32_t l = 0;
    while (((uint64_t)1 << l) < C)
        ++l;
    b.cdiv.shift = 31 + l;
    b.cdiv.m = (uint32_t)((((uint64_t)1 << (31 + l)) + C - 1) / C);
    if (g)
        *g = b;
    return true;
}

unsigned lds_eval_blocks()
{
    // one workgroup per compute unit of the current device (256 on MI355X)
    static int cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (cus[dev] <= 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        cus[dev] = c;
    }
    return (unsigned)cus[dev];
}

size_t bucket_bytes(const BucketGeom &g)
{
    return (size_t)g.ranges * g.region * 4 + (size_t)g.ranges * g.NJ * 8 +
           (size_t)g.ranges * 8 + kXcds * 8 + 1280;
}

uint64_t sample_tag(int64_t n, int64_t m, uint64_t seed, uint32_t bshift, uint32_t layout)
{
    // splitmix64 finaliser over the arguments that fix the records and where
    // they sit
    uint64_t h = 0x9E3779B97F4A7C15ull;
    const uint64_t parts[5] = {(uint64_t)n, (uint64_t)m, seed, (uint64_t)bshift, (uint64_t)layout};
    for (uint64_t v : parts) {
        h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h ^= h >> 30;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 27;
        h *= 0x94D049BB133111EBull;
        h ^= h >> 31;
    }
    return h | 1ull;
}

hipError_t launch_bucket_generate(const Inst &I, const BucketGeom &B, hipStream_t st)
{
    if (B.ranges > 0x7FFFFFFFull || B.NJ > kMaxPartnerBlocks)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bkt_prepare, dim3(1), dim3(64), 0, st, B, 1);
    const size_t lds = ((size_t)kRangeSlots + 2 * (size_t)B.NJ) * sizeof(uint32_t);
    if (I.inv_nf != 0.0f && I.n < (1u << 24))
        hipLaunchKernelGGL(k_bkt_generate<2>, dim3((unsigned)B.ranges), dim3(kGenThreads), lds,
                           st, I, B);
    else if (I.inv_nf != 0.0f)
        hipLaunchKernelGGL(k_bkt_generate<1>, dim3((unsigned)B.ranges), dim3(kGenThreads), lds,
                           st, I, B);
    else
        hipLaunchKernelGGL(k_bkt_generate<0>, dim3((unsigned)B.ranges), dim3(kGenThreads), lds,
                           st, I, B);
    hipLaunchKernelGGL(k_bkt_seal, dim3(1), dim3(64), 0, st, B);
    return hipGetLastError();
}

static hipError_t prepare_eval(const Inst &I, const BucketGeom &B, bool reuse, hipStream_t st)
{
    if (!reuse) {
        const hipError_t e = launch_bucket_generate(I, B, st);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_bkt_prepare, dim3(1), dim3(64), 0, st, B, 0);
    return hipGetLastError();
}

hipError_t launch_bucket_plain(const Inst &I, const BucketGeom &B0, const PassAShape &sh,
                               bool reuse, hipStream_t st)
{
    const BucketGeom B = eval_geom(I, B0);
    hipError_t e = prepare_eval(I, B, reuse, st);
    if (e != hipSuccess)
        return e;
    if (I.sim.kind == kSimDot)
        return launch_bucket_eval<kSimDot>(I, B, sh, st);
    if (I.sim.kind == kSimCos)
        return launch_bucket_eval<kSimCos>(I, B, sh, st);
    return launch_bucket_eval<kSimNone>(I, B, sh, st);
}

hipError_t launch_bucket_sweep(const Inst &I, const SweepArgs &S, const BucketGeom &B0,
                               const PassAShape &sh, hipStream_t st)
{
    const BucketGeom B = eval_geom(I, B0);
    hipError_t e = prepare_eval(I, B, false, st);
    if (e != hipSuccess)
        return e;
    return launch_bucket_eval_sweep(I, S, B, sh, st);
}

}  // namespace sng
