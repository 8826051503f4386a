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

#include "sng_pass_a.hpp"

namespace sng {

constexpr uint32_t kRecOffShift = 18;  // record: call offset (14 bits) | word (2) | partner (16)

// Decisions take point indices; row pointers for the binary64 recheck are
// formed only inside the band. record() receives the slot's global call
// number as a functor, evaluated only for accepted slots. kSim: the
// instance's similarity query instead of the distance (per-pair band on the
// same binary32 distance).
template <bool kSim>
struct BucketPlainPolicy {
    int out_deg;  // 1: out-degrees (no partner-side count)
    const float *X;
    int64_t ld;
    int d;
    uint32_t *deg;
    uint32_t *mask;
    float lo, hi;
    double eps2;
    SimQuery sim;

    __device__ __forceinline__ int decide(float F, uint32_t i, uint32_t j, Tally &t, int q)
    {
        if constexpr (kSim) {
            const int r = sim.band(i, j, F);
            if (r >= 0)
                return r;
            t.rechecked += (q == 0);
            return sim_accept_f64(X + (int64_t)i * ld, X + (int64_t)j * ld, d, sim.kind, sim.tau);
        } else {
            if (F <= lo)
                return 1;
            if (F > hi)
                return 0;
            t.rechecked += (q == 0);
            return sqdist_f64(X + (int64_t)i * ld, X + (int64_t)j * ld, d) <= eps2;
        }
    }
    template <class CallFn>
    __device__ __forceinline__ void record(int acc, uint32_t i, uint32_t j, CallFn call_of, int w,
                                           int q, Tally &t)
    {
        if (acc && q == 0) {
            const uint64_t call = call_of();
            atomicAdd(deg + i, 1u);
            if (!out_deg)
                atomicAdd(deg + j, 1u);
            atomicOr(mask + (call >> 3), 1u << (4 * (call & 7) + w));
            t.accepted += 1;
        }
    }
};

struct BucketSweepPolicy {
    int out_deg;  // 1: out-degrees (no partner-side count)
    const float *X;
    int64_t ld;
    int d;
    uint32_t *hist;
    uint8_t *codes;  // byte per slot (call*4 + word), pre-filled with K
    const float *lo;
    const float *hi;
    const double *e2;
    int K;
    float hi_max;

    __device__ __forceinline__ int decide(float F, uint32_t i, uint32_t j, Tally &t, int q)
    {
        if (!(F <= hi_max))
            return K;
        int a = 0, b = K - 1;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (F <= hi[mid])
                b = mid;
            else
                a = mid + 1;
        }
        if (F <= lo[a])
            return a;
        t.rechecked += (q == 0);
        const double D = sqdist_f64(X + (int64_t)i * ld, X + (int64_t)j * ld, d);
        int k = a;
        while (k < K && !(D <= e2[k]))
            ++k;
        return k;
    }
    template <class CallFn>
    __device__ __forceinline__ void record(int b, uint32_t i, uint32_t j, CallFn call_of, int w,
                                           int q, Tally &t)
    {
        if (b < K && q == 0) {
            const uint64_t call = call_of();
            atomicAdd(hist + (uint64_t)i * K + b, 1u);
            if (!out_deg)
                atomicAdd(hist + (uint64_t)j * K + b, 1u);
            codes[call * 4ull + (uint64_t)w] = (uint8_t)b;
            t.accepted += 1;
        }
    }
};

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

__global__ __launch_bounds__(kGenThreads) void k_bkt_generate(Inst I, BucketGeom B)
{
    extern __shared__ uint32_t lds_u32[];
    __shared__ uint32_t wsum[kGenThreads / kWave];
    uint32_t *stage = lds_u32;              // [kRangeSlots]
    uint32_t *cnt = lds_u32 + kRangeSlots;  // [NJ]
    uint32_t *pre = cnt + B.NJ;             // [NJ]
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
    // key: partner block << 16 | rank of the record within its block
    uint32_t key[4 * kCallsPerThread], rec[4 * kCallsPerThread];
    uint32_t self = 0;
#pragma unroll
    for (uint32_t c = 0; c < kCallsPerThread; ++c) {
        const uint32_t off = c * kGenThreads + tid;
        const bool live = call_lo + off < call_hi;
        uint32_t cc = c0 + off, ii = i0;
        if (cc >= I.C) {
            const uint32_t q = div_exact(cc, I.C, I.inv_C);
            ii += q;
            cc -= q * I.C;
        }
        const uint32_t nvalid = live ? min(4u, I.m - 4u * cc) : 0u;
        const Words4 W = philox10(cc, ii, I.key0, I.key1);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint32_t kk = ~0u, rr = 0;
            if ((uint32_t)w < nvalid) {
                const uint32_t j = mod_exact(W.w[w], I.n, I.inv_n);
                if (j == ii) {
                    ++self;
                } else {
                    const uint32_t J = j >> B.bshift;
                    kk = (J << 16) | atomicAdd(cnt + J, 1u);
                    rr = (off << kRecOffShift) | ((uint32_t)w << 16) |
                         (j & ((1u << B.bshift) - 1u));
                }
            }
            key[4 * c + w] = kk;
            rec[4 * c + w] = rr;
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
    for (uint32_t k = 4 * tid; k < total; k += 4 * kGenThreads) {
        if (k + 4 <= total) {
            *reinterpret_cast<uint4 *>(dst + k) = *reinterpret_cast<const uint4 *>(stage + k);
        } else {
            for (uint32_t e = k; e < total; ++e)
                dst[e] = stage[e];
        }
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

// Every evaluate kernel starts here: false (and one count in the overflow
// counter) when the workspace does not hold the sample of B.tag, so a stale
// or missing sample is reported instead of read. Uniform over the grid.
__device__ __forceinline__ bool sample_ok(const Inst &I, const BucketGeom &B)
{
    const unsigned long long have = B.hdr[0];
    if (have != B.tag) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicAdd(I.cnt + kCntOverflow, 1ull);
        return false;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(I.cnt + kCntSelf, B.hdr[1]);
    return true;
}

// ---------------------------------------------------------------------------
// Evaluate.
// ---------------------------------------------------------------------------
// One work item (ticket): the segments of partner block J from kTicketRanges
// consecutive generator ranges, walked as one sequence of records f =
// 0..total-1. Lane l < T holds the segment of range r0 + l (its record base,
// first record index in the sequence, and first source and call). The groups
// of the wave take the records interleaved (record f goes to group f mod
// kGroups), so every record load is a coalesced read; a window of P*kGroups
// records meets only a few segments, found with wave-wide ballots and
// scalar reads of those segments' entries. Records of the next window are
// loaded while the current one is decided.
constexpr uint32_t kTicketRanges = 16;
static_assert(kTicketRanges <= kWave, "one lane per segment of a ticket");

template <class Row, int OB, bool kBuf, class Pol>
__device__ __forceinline__ void eval_ticket(const Inst &I, const BucketGeom &B, Pol &pol,
                                            uint64_t r0, uint32_t T, uint32_t J, Tally &tally)
{
    constexpr int G = Row::kG;
    constexpr int P = 4 * OB;  // records in flight per group
    constexpr int kGroups = kWave / G;
    constexpr uint32_t kStep = (uint32_t)P * kGroups;
    const int lane = lane_id();
    const int q = lane & (G - 1);
    const int grp = lane / G;
    // Records of the ticket: T consecutive regions of the record array, read
    // through a buffer descriptor with 32-bit offsets.
    const __amdgpu_buffer_rsrc_t rrec =
        buf_rsrc(B.rec + r0 * B.region, (uint32_t)(T * B.region * sizeof(uint32_t)));
    uint32_t cnt_l = 0, i0_l = 0, c0_l = 0, base_l = 0;
    if ((uint32_t)lane < T) {
        const uint64_t r = r0 + (uint64_t)lane;
        base_l = (uint32_t)lane * (uint32_t)B.region + B.seg[(r * B.NJ + J) * 2 + 0];
        cnt_l = B.seg[(r * B.NJ + J) * 2 + 1];
        i0_l = B.start[2 * r + 0];
        c0_l = B.start[2 * r + 1];
    }
    uint32_t incl = cnt_l;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const uint32_t u = __shfl_up(incl, s);
        if (lane >= s)
            incl += u;
    }
    const uint32_t excl_l = incl - cnt_l;  // non-decreasing over the lanes
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    if (total == 0)
        return;  // wave-uniform
    // record f of segment l < T sits at index base_l + f of the ticket's
    // records (no wrap: excl_l <= l * region)
    base_l -= excl_l;

    // Loads the records of window [f0, f0 + kStep) and their segments.
    auto locate = [&](uint32_t f0, uint32_t (&vv)[P], uint32_t (&ss)[P]) {
        const int s_lo = __popcll(__ballot(excl_l <= f0)) - 1;
        const int s_hi = min(__popcll(__ballot(excl_l < f0 + kStep)), (int)T) - 1;
        uint32_t bk[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            bk[k] = (uint32_t)__builtin_amdgcn_readlane((int)base_l, s_lo);
            ss[k] = (uint32_t)s_lo;
        }
        for (int b = s_lo + 1; b <= s_hi; ++b) {  // wave-uniform
            const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)excl_l, b);
            const uint32_t bb = (uint32_t)__builtin_amdgcn_readlane((int)base_l, b);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if (f0 + (uint32_t)(k * kGroups + grp) >= e) {
                    bk[k] = bb;
                    ss[k] = (uint32_t)b;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint32_t f = f0 + (uint32_t)(k * kGroups + grp);
            vv[k] = (f < total)
                        ? __builtin_amdgcn_raw_buffer_load_b32(rrec, (int)((bk[k] + f) * 4u), 0, 0)
                        : 0u;
        }
    };

    const uint32_t jbase = J << B.bshift;
    const float *__restrict__ X = I.X;
    const int64_t ld = I.ld;
    const int d = I.d;
    const uint32_t ld4 = (uint32_t)ld * 4u;  // row stride in bytes (buffer form)
    __amdgpu_buffer_rsrc_t rs;
    if constexpr (kBuf)
        rs = buf_rsrc(X, B.x_bytes);
    uint32_t nv[P], ns[P];
    locate(0, nv, ns);
    for (uint32_t f0 = 0; f0 < total; f0 += kStep) {  // wave-uniform
        uint32_t v[P], sv[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            v[k] = nv[k];
            sv[k] = ns[k];
        }
        if (f0 + kStep < total)
            locate(f0 + kStep, nv, ns);
        uint32_t ii[P], cj[P];
        bool live[P];
        typename Row::Buf bi[P], bj[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            live[k] = f0 + (uint32_t)(k * kGroups + grp) < total;  // group-uniform
            const uint32_t i0 = (uint32_t)__shfl((int)i0_l, (int)sv[k]);
            const uint32_t c0 = (uint32_t)__shfl((int)c0_l, (int)sv[k]);
            const uint32_t co = v[k] >> kRecOffShift;
            cj[k] = jbase | (v[k] & 0xFFFFu);
            ii[k] = i0 + div_magic(c0 + co, B.cdiv);
            if (live[k] && !(ii[k] < I.n && cj[k] < I.n)) {  // never for a valid sample
                live[k] = false;
                if (q == 0)
                    atomicAdd(I.cnt + kCntOverflow, 1ull);
            }
            const uint32_t sj = live[k] ? cj[k] : 0u;  // row 0 always exists
            const uint32_t si = live[k] ? ii[k] : 0u;
            if constexpr (kBuf) {
                bj[k] = Row::fetchb(rs, __umul24(sj, ld4), q, d);
                bi[k] = Row::fetchb(rs, __umul24(si, ld4), q, d);
            } else {
                bj[k] = Row::fetch(X + (int64_t)sj * ld, q, d);
                bi[k] = Row::fetch(X + (int64_t)si * ld, q, d);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (!live[k])
                continue;
            float F = group_sum<G>(Row::partial2(bi[k], bj[k], q, d));
            F = __int_as_float((int)group_bcast<G>((uint32_t)__float_as_int(F), 0));
            const int res = pol.decide(F, ii[k], cj[k], tally, q);
            const uint32_t vk = v[k], sk = sv[k];
            pol.record(res, ii[k], cj[k],
                       [&]() { return (r0 + sk) * kRangeCalls + (vk >> kRecOffShift); },
                       (int)((vk >> 16) & 3u), q, tally);
        }
    }
}

// XCD this wavefront runs on (hardware register XCC_ID, 4 bits).
__device__ __forceinline__ uint32_t my_xcd()
{
    return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % kXcds;
}

// Each XCD owns the partner blocks J = x, x + kXcds, ... and a queue over
// (J, ticket) in block-major order: all wavefronts of the XCD work on one
// partner block at a time (kept in that XCD's L2) while the source rows
// stream in sequential pieces. Wavefronts then help the other queues until
// all are empty, so every ticket is taken exactly once whichever XCDs the
// workgroups land on.
template <class Row, int OB, bool kBuf, class Pol>
__device__ __forceinline__ void eval_all(const Inst &I, const BucketGeom &B, Pol &pol,
                                         Tally &tally)
{
    const uint32_t home = my_xcd();
    const uint64_t tpj = (B.ranges + kTicketRanges - 1) / kTicketRanges;  // tickets per block
    for (uint32_t s = 0; s < kXcds; ++s) {
        const uint32_t x = (home + s) % kXcds;
        const uint64_t blocks = (B.NJ > x) ? (B.NJ - x + kXcds - 1) / kXcds : 0;
        const uint64_t total = blocks * tpj;
        for (;;) {
            unsigned long long got = 0;
            if (lane_id() == 0)
                got = atomicAdd(B.queue + x, 1ull);
            // lane 0's ticket, held in scalar registers (uniform to the compiler)
            const uint64_t e =
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(got >> 32))
                 << 32) |
                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
            if (e >= total)
                break;  // wave-uniform
            const uint64_t jl = e / tpj;
            const uint64_t r0 = (e - jl * tpj) * kTicketRanges;
            const uint64_t left = B.ranges - r0;
            const uint32_t T = (uint32_t)(left < kTicketRanges ? left : kTicketRanges);
            eval_ticket<Row, OB, kBuf>(I, B, pol, r0, T, (uint32_t)(x + jl * kXcds), tally);
        }
    }
}

template <class Row, int OB, bool kBuf, bool kSim>
__global__ __launch_bounds__(256) void k_bkt_eval_plain(Inst I, BucketGeom B)
{
    if (!sample_ok(I, B))
        return;
    BucketPlainPolicy<kSim> pol;
    pol.out_deg = I.out_deg;
    pol.X = I.X;
    pol.ld = I.ld;
    pol.d = I.d;
    pol.deg = I.deg;
    pol.mask = I.mask;
    pol.lo = I.lo;
    pol.hi = I.hi;
    pol.eps2 = I.eps2;
    pol.sim = I.sim;
    Tally t;
    eval_all<Row, OB, kBuf>(I, B, pol, t);
    commit_tally(t, I.cnt);
}

template <class Row, int OB, bool kBuf>
__global__ __launch_bounds__(256) void k_bkt_eval_sweep(Inst I, BucketGeom B, SweepArgs S)
{
    if (!sample_ok(I, B))
        return;
    __shared__ float s_lo[kSweepMaxK], s_hi[kSweepMaxK];
    __shared__ double s_e2[kSweepMaxK];
    for (int k = threadIdx.x; k < S.K; k += blockDim.x) {
        s_lo[k] = S.c.lo[k];
        s_hi[k] = S.c.hi[k];
        s_e2[k] = S.c.e2[k];
    }
    __syncthreads();
    BucketSweepPolicy pol;
    pol.out_deg = I.out_deg;
    pol.X = I.X;
    pol.ld = I.ld;
    pol.d = I.d;
    pol.hist = S.hist;
    pol.codes = reinterpret_cast<uint8_t *>(S.codes);
    pol.lo = s_lo;
    pol.hi = s_hi;
    pol.e2 = s_e2;
    pol.K = S.K;
    pol.hi_max = S.c.hi[S.K - 1];
    Tally t;
    eval_all<Row, OB, kBuf>(I, B, pol, t);
    commit_tally(t, I.cnt);
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
    // partner block: at most 2^16 rows and about half a MB of rows
    int bs = 16;
    while (bs > 6 && ((uint64_t)1 << bs) * (uint64_t)d * 4 > (512u << 10))
        --bs;
    b.bshift = (uint32_t)bs;
    b.NJ = (uint32_t)((n + ((int64_t)1 << bs) - 1) >> bs);
    if (b.NJ > kMaxPartnerBlocks)
        return false;
    const uint64_t C = (uint64_t)((m + 3) / 4);
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
    hipLaunchKernelGGL(k_bkt_generate, dim3((unsigned)B.ranges), dim3(kGenThreads),
                       ((size_t)kRangeSlots + 2 * (size_t)B.NJ) * sizeof(uint32_t), st, I, B);
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

// Rows are read through a buffer descriptor with 32-bit byte offsets formed
// by 24-bit multiplies when X spans less than 4 GB, the row index fits 24
// bits and the row stride in bytes fits 24 bits.
static bool use_buffer(const Inst &I)
{
    const uint64_t bytes = (uint64_t)I.n * (uint64_t)I.ld * 4u;
    return bytes < ((uint64_t)1 << 32) - 4096 && I.n < (1u << 24) &&
           (uint64_t)I.ld * 4u < ((uint64_t)1 << 24);
}

static unsigned eval_blocks(const BucketGeom &B)
{
    // 128 blocks of 4 waves per XCD (four per CU), a multiple of kXcds
    (void)B;
    return kXcds * 128;
}

// The geometry as the evaluate kernels take it: with the byte span of X for
// the buffer form.
static BucketGeom eval_geom(const Inst &I, const BucketGeom &B)
{
    BucketGeom g = B;
    g.x_bytes = use_buffer(I) ? (uint32_t)((uint64_t)I.n * (uint64_t)I.ld * 4u) : 0u;
    return g;
}

hipError_t launch_bucket_plain(const Inst &I, const BucketGeom &B0, const PassAShape &sh,
                               bool reuse, hipStream_t st)
{
    const BucketGeom B = eval_geom(I, B0);
    hipError_t e = prepare_eval(I, B, reuse, st);
    if (e != hipSuccess)
        return e;
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t) -> hipError_t {
        if constexpr (Row::kPrefetch) {
            const bool buf = use_buffer(I), sim = I.sim.kind != kSimNone;
            if (buf && !sim)
                hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB, true, false>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B);
            else if (!sim)
                hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB, false, false>),
                                   dim3(eval_blocks(B)), dim3(256), 0, st, I, B);
            else if (buf)
                hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB, true, true>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B);
            else
                hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB, false, true>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

hipError_t launch_bucket_sweep(const Inst &I, const SweepArgs &S, const BucketGeom &B0,
                               const PassAShape &sh, hipStream_t st)
{
    const BucketGeom B = eval_geom(I, B0);
    hipError_t e = prepare_eval(I, B, false, st);
    if (e != hipSuccess)
        return e;
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t) -> hipError_t {
        if constexpr (Row::kPrefetch) {
            if (use_buffer(I))
                hipLaunchKernelGGL((k_bkt_eval_sweep<Row, OB, true>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B, S);
            else
                hipLaunchKernelGGL((k_bkt_eval_sweep<Row, OB, false>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B, S);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

}  // namespace sng
