// Sampled-distance pass scheduled for L2 reuse.
//
// Sample slots are uniform over all partners, so a direct gather reads one
// random row of X per slot; rows narrower than an L2 line (128 B) waste the
// rest of the line, and none is reused. This schedule first sorts the slots
// by partner block and then evaluates them block by block:
//
//   generate  one wavefront per range of kGenCalls Philox calls. It counts
//             its non-self slots per partner block (2^bshift rows, about half
//             a MB of X), then regenerates them and writes 4-byte records
//             (call offset in its range, word, partner offset in the block)
//             into one segment per block of its private region;
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
constexpr uint64_t kTicket = 4;        // consecutive segments taken per queue atomic

struct BucketPlainPolicy {
    uint32_t *deg;
    uint32_t *mask;
    float lo, hi;
    double eps2;

    __device__ __forceinline__ int decide(float F, const float *rowi, const float *rowj, int d,
                                          Tally &t, int q)
    {
        if (F <= lo)
            return 1;
        if (F > hi)
            return 0;
        t.rechecked += (q == 0);
        return sqdist_f64(rowi, rowj, d) <= eps2;
    }
    __device__ __forceinline__ void record(int acc, uint32_t i, uint32_t j, uint64_t call, int w,
                                           int q, Tally &t)
    {
        if (acc) {
            if (q == 0) {
                atomicAdd(deg + i, 1u);
                atomicAdd(deg + j, 1u);
                atomicOr(mask + (call >> 3), 1u << (4 * (call & 7) + w));
                t.accepted += 1;
            }
        }
    }
};

struct BucketSweepPolicy {
    uint32_t *hist;
    uint8_t *codes;  // byte per slot (call*4 + word), pre-filled with K
    const float *lo;
    const float *hi;
    const double *e2;
    int K;
    float hi_max;

    __device__ __forceinline__ int decide(float F, const float *rowi, const float *rowj, int d,
                                          Tally &t, int q)
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
        const double D = sqdist_f64(rowi, rowj, d);
        int k = a;
        while (k < K && !(D <= e2[k]))
            ++k;
        return k;
    }
    __device__ __forceinline__ void record(int b, uint32_t i, uint32_t j, uint64_t call, int w,
                                           int q, Tally &t)
    {
        if (b < K && q == 0) {
            atomicAdd(hist + (uint64_t)i * K + b, 1u);
            atomicAdd(hist + (uint64_t)j * K + b, 1u);
            codes[call * 4ull + (uint64_t)w] = (uint8_t)b;
            t.accepted += 1;
        }
    }
};

// ---------------------------------------------------------------------------
// Generate: count per partner block, prefix, regenerate and scatter records.
// LDS: two counters per block for each of the 4 wavefronts.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bkt_generate(Inst I, BucketGeom B)
{
    extern __shared__ uint32_t lds_u32[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    uint32_t *cnt = lds_u32 + (size_t)wib * 2 * B.NJ;
    uint32_t *cur = cnt + B.NJ;
    const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    uint32_t self = 0;
    if (gw < B.gen_waves) {  // wave-uniform
        for (uint32_t k = lane; k < B.NJ; k += kWave)
            cnt[k] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint64_t call_lo = gw * kGenCalls;
        const uint64_t call_hi = min(call_lo + kGenCalls, I.calls);
        const uint32_t i0 = (uint32_t)(call_lo / I.C);
        const uint32_t c0 = (uint32_t)(call_lo - (uint64_t)i0 * I.C);
        if (lane == 0) {
            B.start[2 * gw + 0] = i0;  // source and call of the range's first call
            B.start[2 * gw + 1] = c0;
        }
        for (int pass = 0; pass < 2; ++pass) {
            for (uint64_t base = call_lo; base < call_hi; base += kWave) {
                const uint32_t off = (uint32_t)(base - call_lo) + (uint32_t)lane;
                const bool live = base + lane < call_hi;
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
                    if ((uint32_t)w < nvalid) {
                        const uint32_t j = mod_exact(W.w[w], I.n, I.inv_n);
                        if (j == ii) {
                            self += (pass == 0);
                        } else {
                            const uint32_t J = j >> B.bshift;
                            if (pass == 0) {
                                atomicAdd(cnt + J, 1u);
                            } else {
                                const uint32_t pos = atomicAdd(cur + J, 1u);
                                B.rec[gw * B.region + pos] = (off << kRecOffShift) |
                                                             ((uint32_t)w << 16) |
                                                             (j & ((1u << B.bshift) - 1u));
                            }
                        }
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (pass == 0) {
                // exclusive prefix of the block counts (lane 0; NJ <= 1024)
                if (lane == 0) {
                    uint32_t run = 0;
                    for (uint32_t k = 0; k < B.NJ; ++k) {
                        const uint32_t c = cnt[k];
                        B.seg[(gw * B.NJ + k) * 2 + 0] = run;
                        B.seg[(gw * B.NJ + k) * 2 + 1] = c;
                        cur[k] = run;
                        run += c;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
    const int slots[1] = {kCntSelf};
    const uint32_t v[1] = {self};
    block_count_add<1>(I.cnt, slots, v);
}

// ---------------------------------------------------------------------------
// Evaluate.
// ---------------------------------------------------------------------------
// One segment: the groups of the wave take its records interleaved (record
// r goes to group r mod kGroups), so every record load is one coalesced read
// of consecutive records; the source and partner rows of P records per group
// are fetched together, then decided one by one.
template <class Row, int OB, class Pol>
__device__ __forceinline__ void eval_segment(const Inst &I, const BucketGeom &B, Pol &pol,
                                             uint64_t gw, uint32_t J, Tally &tally)
{
    constexpr int G = Row::kG;
    constexpr int P = 4 * OB;  // records in flight per group
    constexpr int kGroups = kWave / G;
    const int lane = lane_id();
    const int q = lane & (G - 1);
    const int grp = lane / G;
    const uint32_t off = B.seg[(gw * B.NJ + J) * 2 + 0];
    const uint32_t cnt = B.seg[(gw * B.NJ + J) * 2 + 1];
    if (cnt == 0)
        return;
    const uint32_t *rec = B.rec + gw * B.region + off;
    const uint64_t call_lo = gw * kGenCalls;
    const uint32_t i0 = B.start[2 * gw + 0];
    const uint32_t c0 = B.start[2 * gw + 1];
    const uint32_t jbase = J << B.bshift;
    const float *__restrict__ X = I.X;
    const int64_t ld = I.ld;
    const int d = I.d;
    constexpr uint32_t kStep = (uint32_t)P * kGroups;
    uint32_t nxt[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const uint32_t r = k * kGroups + grp;
        nxt[k] = (r < cnt) ? rec[r] : 0u;
    }
    for (uint32_t r0 = 0; r0 < cnt; r0 += kStep) {  // wave-uniform
        uint32_t v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            v[k] = nxt[k];
            const uint32_t r = r0 + kStep + k * kGroups + grp;
            nxt[k] = (r < cnt) ? rec[r] : 0u;
        }
        uint32_t ii[P], cj[P], ww[P];
        uint64_t call[P];
        bool live[P];
        typename Row::Buf bi[P], bj[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            live[k] = r0 + k * kGroups + grp < cnt;  // group-uniform
            const uint32_t co = v[k] >> kRecOffShift;
            ww[k] = (v[k] >> 16) & 3u;
            cj[k] = jbase | (v[k] & 0xFFFFu);
            uint32_t cc = c0 + co, i = i0;
            if (cc >= I.C) {
                const uint32_t qq = div_exact(cc, I.C, I.inv_C);
                i += qq;
                cc -= qq * I.C;
            }
            ii[k] = i;
            call[k] = call_lo + co;
            const uint32_t sj = live[k] ? cj[k] : 0u;  // row 0 always exists
            const uint32_t si = live[k] ? i : 0u;
            bj[k] = Row::fetch(X + (int64_t)sj * ld, q, d);
            bi[k] = Row::fetch(X + (int64_t)si * ld, q, d);
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (!live[k])
                continue;
            float F = group_sum<G>(Row::partial2(bi[k], bj[k], q, d));
            F = __int_as_float((int)group_bcast<G>((uint32_t)__float_as_int(F), 0));
            const int res = pol.decide(F, X + (int64_t)ii[k] * ld, X + (int64_t)cj[k] * ld, d,
                                       tally, q);
            pol.record(res, ii[k], cj[k], call[k], (int)ww[k], q, tally);
        }
    }
}

// XCD this wavefront runs on (hardware register XCC_ID, 4 bits).
__device__ __forceinline__ uint32_t my_xcd()
{
    return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % kXcds;
}

// Each XCD owns the partner blocks J = x, x + kXcds, ... and a queue over
// (J, generator range) in block-major order: all wavefronts of the XCD work
// on one partner block at a time (kept in that XCD's L2) while the source
// rows stream in small sequential pieces. Wavefronts take kTicket
// consecutive segments per queue atomic, then help the other queues until
// all are empty, so every segment is taken exactly once whichever XCDs the
// workgroups land on.
template <class Row, int OB, class Pol>
__device__ __forceinline__ void eval_all(const Inst &I, const BucketGeom &B, Pol &pol,
                                         Tally &tally)
{
    const uint32_t home = my_xcd();
    for (uint32_t s = 0; s < kXcds; ++s) {
        const uint32_t x = (home + s) % kXcds;
        const uint64_t blocks = (B.NJ > x) ? (B.NJ - x + kXcds - 1) / kXcds : 0;
        const uint64_t total = blocks * B.gen_waves;
        for (;;) {
            unsigned long long e0 = 0;
            if (lane_id() == 0)
                e0 = atomicAdd(B.queue + x, (unsigned long long)kTicket);
            e0 = __shfl(e0, 0);
            if (e0 >= total)
                break;  // wave-uniform
            const uint64_t e1 = min(e0 + kTicket, total);
            for (uint64_t e = e0; e < e1; ++e) {
                const uint64_t jl = e / B.gen_waves;
                const uint64_t gw = e - jl * B.gen_waves;
                eval_segment<Row, OB>(I, B, pol, gw, (uint32_t)(x + jl * kXcds), tally);
            }
        }
    }
}

template <class Row, int OB>
__global__ __launch_bounds__(256) void k_bkt_eval_plain(Inst I, BucketGeom B)
{
    BucketPlainPolicy pol;
    pol.deg = I.deg;
    pol.mask = I.mask;
    pol.lo = I.lo;
    pol.hi = I.hi;
    pol.eps2 = I.eps2;
    Tally t;
    eval_all<Row, OB>(I, B, pol, t);
    commit_tally(t, I.cnt);
}

template <class Row, int OB>
__global__ __launch_bounds__(256) void k_bkt_eval_sweep(Inst I, BucketGeom B, SweepArgs S)
{
    __shared__ float s_lo[kSweepMaxK], s_hi[kSweepMaxK];
    __shared__ double s_e2[kSweepMaxK];
    for (int k = threadIdx.x; k < S.K; k += blockDim.x) {
        s_lo[k] = S.c.lo[k];
        s_hi[k] = S.c.hi[k];
        s_e2[k] = S.c.e2[k];
    }
    __syncthreads();
    BucketSweepPolicy pol;
    pol.hist = S.hist;
    pol.codes = reinterpret_cast<uint8_t *>(S.codes);
    pol.lo = s_lo;
    pol.hi = s_hi;
    pol.e2 = s_e2;
    pol.K = S.K;
    pol.hi_max = S.c.hi[S.K - 1];
    Tally t;
    eval_all<Row, OB>(I, B, pol, t);
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
    b.gen_waves = (calls + kGenCalls - 1) / kGenCalls;
    b.region = kGenCalls * 4;
    if (g)
        *g = b;
    return true;
}

size_t bucket_bytes(const BucketGeom &g)
{
    return (size_t)g.gen_waves * g.region * 4 + (size_t)g.gen_waves * g.NJ * 8 +
           (size_t)g.gen_waves * 8 + kXcds * 8 + 1280;
}

static hipError_t generate(const Inst &I, const BucketGeom &B, hipStream_t st)
{
    hipError_t e0 = launch_fill_u64(B.queue, kXcds, 0ull, st);
    if (e0 != hipSuccess)
        return e0;
    const uint64_t blocks = (B.gen_waves + 3) / 4;
    if (blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bkt_generate, dim3((unsigned)blocks), dim3(256),
                       (size_t)B.NJ * 2 * 4 * sizeof(uint32_t), st, I, B);
    return hipGetLastError();
}

static unsigned eval_blocks(const BucketGeom &B)
{
    // 128 blocks of 4 waves per XCD (four per CU), a multiple of kXcds
    (void)B;
    return kXcds * 128;
}

hipError_t launch_bucket_plain(const Inst &I, const BucketGeom &B, const PassAShape &sh,
                               hipStream_t st)
{
    hipError_t e = generate(I, B, st);
    if (e != hipSuccess)
        return e;
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t) -> hipError_t {
        if constexpr (Row::kPrefetch) {
            hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB>), dim3(eval_blocks(B)), dim3(256), 0, st,
                               I, B);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

hipError_t launch_bucket_sweep(const Inst &I, const SweepArgs &S, const BucketGeom &B,
                               const PassAShape &sh, hipStream_t st)
{
    hipError_t e = generate(I, B, st);
    if (e != hipSuccess)
        return e;
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t) -> hipError_t {
        if constexpr (Row::kPrefetch) {
            hipLaunchKernelGGL((k_bkt_eval_sweep<Row, OB>), dim3(eval_blocks(B)), dim3(256), 0, st,
                               I, B, S);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

}  // namespace sng
