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
#include <math.h>
#include <string.h>

#include "sng_bucket_eval.hpp"

namespace sng {


// ---------------------------------------------------------------------------
// Generate. LDS: a count and an offset per partner block, then the record
// stage of the range.
// ---------------------------------------------------------------------------
constexpr uint32_t kGenThreads = 1024;
constexpr uint32_t kCallsPerThread = (uint32_t)kRangeCalls / kGenThreads;
constexpr uint32_t kRangeSlots = 4 * (uint32_t)kRangeCalls;
static_assert(kCallsPerThread * kGenThreads == kRangeCalls, "range split");
static_assert(kRangeCalls <= (1u << (32 - kRecOffShift)), "call offset field");
static_assert(kMaxPartnerBlocks <= kGenThreads, "one count per thread in the prefix");

// Exclusive prefix of v over a workgroup of kGenThreads threads; *total gets
// the sum. Each wavefront scans its values, wavefront 0 then scans the
// wavefront totals. wsum: 2 * kGenWaves + 1 words of LDS.
constexpr int kGenWaves = (int)(kGenThreads / kWave);
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
    if (w == 0) {
        const uint32_t t = lane < kGenWaves ? wsum[lane] : 0u;
        uint32_t y = t;
#pragma unroll
        for (int s = 1; s < kGenWaves; s <<= 1) {
            const uint32_t u = __shfl_up(y, s);
            if (lane >= s)
                y += u;
        }
        if (lane < kGenWaves)
            wsum[kGenWaves + lane] = y - t;
        if (lane == kGenWaves - 1)
            wsum[2 * kGenWaves] = y;
    }
    __syncthreads();
    *total = wsum[2 * kGenWaves];
    return wsum[kGenWaves + w] + x - v;
}

// Record stage layout in LDS: the counts of partner blocks J <= NJ, then
// their offsets (one word each, so consecutive blocks fall in consecutive
// banks), each array rounded up to an even length so that the stage that
// follows is 16-byte aligned. Block NJ collects the slots that make no
// record (self pairs, words past m, calls past the range), so every slot
// takes one unconditional counting step.
__host__ __device__ __forceinline__ uint32_t gen_pairs(uint32_t NJ)
{
    return (NJ + 2u) & ~1u;
}

// kMod: 0 the binary64 remainder, 1 the binary32 one, 2 the binary32 one
// with a 24-bit multiply (n < 2^24), 3 the one-sided binary32 one
// (4096 <= n <= 2^23, inv_lo from gen_inv_lo).
template <int kMod>
__global__ __launch_bounds__(kGenThreads) void k_bkt_generate(Inst I, BucketGeom B, float inv_lo)
{
    extern __shared__ __align__(16) uint32_t lds_u32[];
    __shared__ uint32_t wsum[2 * kGenWaves + 1];
    const uint32_t NJ = B.NJ;
    uint32_t *cnt = lds_u32;                        // [gen_pairs(NJ)]
    uint32_t *pre = lds_u32 + gen_pairs(NJ);        // [gen_pairs(NJ)]
    uint32_t *stage = lds_u32 + 2 * gen_pairs(NJ);  // [kRangeSlots]
    const uint32_t tid = threadIdx.x;
    // Persistent: one workgroup per compute unit walks ranges blockIdx.x,
    // blockIdx.x + gridDim.x, ...; the sorted records of a range are copied
    // out of the stage while the next range is counted (the stage is only
    // written again after that count).
    uint32_t *prev_dst = nullptr;  // the previous range's records, still in the stage
    uint32_t prev_total = 0;
    // This thread's 16-byte piece c of the previous range. The last piece
    // may carry up to three stale words past the records; they land inside
    // the range's own region, where nothing reads them.
    auto copy_piece = [&](uint32_t c) {
        const uint32_t k = 4 * (tid + c * kGenThreads);
        if (k < prev_total)
            *reinterpret_cast<uint4 *>(prev_dst + k) = *reinterpret_cast<const uint4 *>(stage + k);
    };
    static_assert(4 * kGenThreads * kCallsPerThread == kRangeSlots, "one piece per call step");
    for (uint64_t r = blockIdx.x; r < B.ranges; r += gridDim.x) {
        const uint64_t call_lo = r * kRangeCalls;
        const uint64_t call_hi = min(call_lo + kRangeCalls, I.calls);
        const uint32_t ncalls = (uint32_t)(call_hi - call_lo);
        const uint32_t i0 = (uint32_t)(call_lo / I.C);
        const uint32_t c0 = (uint32_t)(call_lo - (uint64_t)i0 * I.C);
        for (uint32_t k = tid; k < gen_pairs(NJ); k += kGenThreads)
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
        // The record's bits above its word and partner fields: the call offset
        // in the range, or for LDS blocks (source offset in the range, call
        // within the point). Both advance by dH per call, and the second by cH
        // more when the call within the point wraps to the next source.
        uint32_t hb, dH, cH;
        const uint32_t w_shift = B.lds ? B.bshift : 16u;
        if (B.lds) {
            const uint32_t s = B.bshift + 2;
            hb = (((ii - i0) << B.tc_bits) | cc) << s;
            dH = ((step_q << B.tc_bits) + step_r) << s;
            cH = ((1u << B.tc_bits) - I.C) << s;
        } else {
            hb = tid << kRecOffShift;
            dH = kGenThreads << kRecOffShift;
            cH = 0;
        }
        // word w of a call is a sample iff 4 cc + w < m; calls past the range
        // get a call index no word passes
        uint32_t thr[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            thr[w] = I.m > (uint32_t)w ? I.m - (uint32_t)w : 0u;
        const uint32_t pmask = (1u << B.bshift) - 1u;
        // key: byte offset of the block's offset word (4 J) << 16 | rank of the record in it
        uint32_t key[4 * kCallsPerThread], rec[4 * kCallsPerThread];
        // kAll: every call of the range is live and has four samples (m is a
        // multiple of 4), so only self pairs make no record
        auto count = [&]<bool kAll>() {
#pragma unroll
            for (uint32_t c = 0; c < kCallsPerThread; ++c) {
                const bool live = kAll || tid < ncalls - min(ncalls, c * kGenThreads);
                const uint32_t cc4 = live ? 4u * cc : 0xFFFFFFF0u;
                const Words4 W = philox10(cc, ii, I.key0, I.key1);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint32_t j = kMod == 3   ? mod_f32_floor(W.w[w], I.n, inv_lo)
                                       : kMod == 2 ? mod_f32_n24(W.w[w], I.n, I.inv_nf)
                                       : kMod == 1 ? mod_f32(W.w[w], I.n, I.inv_nf)
                                                   : mod_exact(W.w[w], I.n, I.inv_n);
                    const bool none = (j == ii) | (!kAll && cc4 >= thr[w]);
                    const uint32_t J = none ? NJ : (j >> B.bshift);
                    const uint32_t rank = atomicAdd(cnt + J, 1u);
                    key[4 * c + w] = (J << 18) | rank;
                    rec[4 * c + w] = (j & pmask) | hb | ((uint32_t)w << w_shift);
                }
                cc += step_r;
                ii += step_q;
                hb += dH;
                if (cc >= I.C) {
                    cc -= I.C;
                    ++ii;
                    hb += cH;
                }
                // two pieces per step in the first half of the count, while few
                // records are held in registers
                if (prev_dst && c < kCallsPerThread / 2) {
                    copy_piece(2 * c);
                    copy_piece(2 * c + 1);
                }
            }
        };
        if (ncalls == kRangeCalls && (I.m & 3u) == 0)
            count.template operator()<true>();
        else
            count.template operator()<false>();
        __syncthreads();
        const uint32_t v = tid < NJ ? cnt[tid] : 0u;
        uint32_t total;
        const uint32_t ex = gen_exclusive(v, wsum, &total);
        if (tid < NJ) {
            pre[tid] = ex;
            *reinterpret_cast<uint2 *>(B.seg + (r * NJ + tid) * 2) = make_uint2(ex, v);
        }
        if (tid == 0) {
            // the slots without a record go past the records
            pre[NJ] = total;
            // self pairs: the range's sample slots (words below m of its calls;
            // the last call of a point has m - 4 (C - 1) of them) less its records
            const uint32_t wraps = (c0 + ncalls) / I.C;  // points whose last call is in the range
            const uint64_t slots = 4ull * ncalls - (uint64_t)(4u * I.C - I.m) * wraps;
            const uint64_t self = slots - total;
            if (self)
                atomicAdd(B.hdr + 1, (unsigned long long)self);
        }
        __syncthreads();
        const char *preb = reinterpret_cast<const char *>(pre);
#pragma unroll
        for (uint32_t k = 0; k < 4 * kCallsPerThread; ++k) {
            const uint32_t base = *reinterpret_cast<const uint32_t *>(preb + (key[k] >> 16));
            stage[base + (key[k] & 0xFFFFu)] = rec[k];
        }
        __syncthreads();
        prev_dst = B.rec + r * B.region;
        prev_total = total;
    }
    if (prev_dst) {
#pragma unroll
        for (uint32_t c = 0; c < kCallsPerThread; ++c)
            copy_piece(c);
    }
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
    // chosen automatically only when X does not fit one XCD's L2; rows as
    // wide as an L2 line (d = 32) included: on 500k x 32 points the partner
    // blocks take the plain pass from 8.4 to 7.9 ms and the 32 x 4 sweep from
    // 11.7 to 10.7 ms
    if (!force && (uint64_t)n * (uint64_t)d * 4 <= ((uint64_t)8 << 20))
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

unsigned compute_units()
{
    // cached per device (256 on MI355X); racing first calls store the same value
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

// The one-sided remainder's inverse: (1/n)(1 - 2^-21) rounded down to
// binary32, or 0 where that remainder does not apply (n outside
// [4096, 2^23]).
static float gen_inv_lo(uint32_t n)
{
    if (n < 4096u || n > (1u << 23))
        return 0.0f;
    const double x = (1.0 / (double)n) * (1.0 - 0x1p-21);
    float v = (float)x;
    if ((double)v > x)
        v = nextafterf(v, 0.0f);
    return v;
}

hipError_t launch_bucket_generate(const Inst &I, const BucketGeom &B, hipStream_t st)
{
    if (B.ranges > 0x7FFFFFFFull || B.NJ > kMaxPartnerBlocks)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bkt_prepare, dim3(1), dim3(64), 0, st, B, 1);
    const size_t lds = ((size_t)kRangeSlots + 2 * (size_t)gen_pairs(B.NJ)) * sizeof(uint32_t);
    const float inv_lo = gen_inv_lo(I.n);
    const unsigned cus = compute_units();
    const dim3 grid((unsigned)(B.ranges < cus ? B.ranges : cus)), block(kGenThreads);
    if (inv_lo != 0.0f)
        hipLaunchKernelGGL(k_bkt_generate<3>, grid, block, lds, st, I, B, inv_lo);
    else if (I.inv_nf != 0.0f && I.n < (1u << 24))
        hipLaunchKernelGGL(k_bkt_generate<2>, grid, block, lds, st, I, B, 0.0f);
    else if (I.inv_nf != 0.0f)
        hipLaunchKernelGGL(k_bkt_generate<1>, grid, block, lds, st, I, B, 0.0f);
    else
        hipLaunchKernelGGL(k_bkt_generate<0>, grid, block, lds, st, I, B, 0.0f);
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
