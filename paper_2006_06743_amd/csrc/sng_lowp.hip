// Mixed-precision sampled-distance pass (bfloat16 / float16 copy on MFMA).
//
// For a source point i and a tile of 16 of its sampled partners, one wave
// forms the 16 dot products v_i . v_j of the 16-bit copy with
// v_mfma_f32_16x16x32_{bf16,f16}: every row of the A operand is v_i (staged
// once per source in LDS), column c of B is the gathered row of partner c,
// so column c of the 16x16 result holds v_i . v_{j_c} (FP32 accumulation of
// exact 16-bit products). With per-row binary64 statistics ||v||^2, ||v|| and
// the rounding radius r = ||x - scale*v||_2, the squared distance of the copy
//     T^2 = scale^2 (||v_i||^2 + ||v_j||^2 - 2 v_i.v_j)
// is known to within a rigorous error Delta, and the triangle inequality
// gives | ||x_i - x_j|| - T | <= r_i + r_j. A pair is accepted or rejected
// only when that interval, widened by the error of the binary64 definition,
// lies entirely on one side of eps; otherwise its slot goes to a queue and a
// second kernel re-decides it with the defining binary64 sum. Degrees and
// accept bits therefore equal those of the plain path exactly.
#include "sng_internal.hpp"

namespace sng {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ double decode(uint16_t b)
{
    if constexpr (PREC == 1) {
        return (double)__uint_as_float((uint32_t)b << 16);
    } else {
        _Float16 h;
        __builtin_memcpy(&h, &b, 2);
        return (double)h;
    }
}

// ---------------------------------------------------------------------------
// Per-row statistics, one wave per row: st[4*i + {0,1,2}] =
// (||v_i||^2, ||v_i||, r_i), each rounded up so that they bound the exact
// values (any summation order: the error terms below cover it).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256) void k_rowstats(Inst I, LowpArgs L)
{
    const int lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const double up = 1.0 + (double)(I.d + 8) * 0x1p-52;
    for (uint64_t i = wave; i < I.n; i += nw) {
        const float *x = I.X + i * I.ld;
        const uint16_t *v = L.Xlp + i * L.ld_lp;
        double nv = 0.0, rr = 0.0;
        for (int k = lane; k < I.d; k += kWave) {
            const double vk = decode<PREC>(v[k]);
            const double e = (double)x[k] - (double)L.scale * vk;
            nv += vk * vk;
            rr += e * e;
        }
        for (int off = 32; off > 0; off >>= 1) {
            nv += __shfl_xor(nv, off);
            rr += __shfl_xor(rr, off);
        }
        if (lane == 0) {
            const double nvu = nv * up;
            const double a = __builtin_sqrt(nvu) * (1.0 + 0x1p-40);
            const double r = __builtin_sqrt(rr * up) * (1.0 + 0x1p-40);
            L.stats[4 * i + 0] = nvu;
            L.stats[4 * i + 1] = a;
            L.stats[4 * i + 2] = r;
            L.stats[4 * i + 3] = 0.0;
        }
    }
}

// The filter's reported bound (not used by any decision): its constants, and
// the largest and summed rounding radii and row norms, reduced by one
// workgroup in a fixed order.
constexpr int kSummaryThreads = 1024;
__global__ __launch_bounds__(kSummaryThreads) void k_rowstats_summary(Inst I, LowpArgs L)
{
    __shared__ double red[4][kSummaryThreads];
    const int t = threadIdx.x;
    double rmax = 0.0, amax = 0.0, rsum = 0.0, asum = 0.0;
    for (uint64_t i = t; i < I.n; i += kSummaryThreads) {
        const double a = L.stats[4 * i + 1], r = L.stats[4 * i + 2];
        rmax = r > rmax ? r : rmax;
        amax = a > amax ? a : amax;
        rsum += r;
        asum += a;
    }
    red[0][t] = rmax;
    red[1][t] = amax;
    red[2][t] = rsum;
    red[3][t] = asum;
    __syncthreads();
    for (int w = kSummaryThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] = red[0][t + w] > red[0][t] ? red[0][t + w] : red[0][t];
            red[1][t] = red[1][t + w] > red[1][t] ? red[1][t + w] : red[1][t];
            red[2][t] += red[2][t + w];
            red[3][t] += red[3][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        double *h = reinterpret_cast<double *>(I.cnt);
        h[kFltGamma] = L.gamma_acc;
        h[kFltGammaNorm] = L.gamma_norm;
        h[kFltScale2] = L.scale2;
        h[kFltEps2] = I.eps2;
        h[kFltRMax] = red[0][0];
        h[kFltAMax] = red[1][0];
        h[kFltRSum] = red[2][0];
        h[kFltASum] = red[3][0];
        I.cnt[kFltRows] = I.n;
    }
}

// 0 reject, 1 accept, 2 undecided. P: FP32 dot of the 16-bit rows.
__device__ __forceinline__ int decide(const LowpArgs &L, float P, double nvi, double ai, double ri,
                                      double nvj, double aj, double rj)
{
    const double E = nvi + nvj - 2.0 * (double)P;
    const double delta = L.gamma_acc * 2.0 * ai * aj + L.gamma_norm * (nvi + nvj) + L.tiny;
    const double s2 = L.scale2;
    const double t2_hi = s2 * (E + delta) * (1.0 + 0x1p-40);
    const double t2_lo = s2 * (E - delta) * (1.0 - 0x1p-40);
    const double R = (ri + rj) * (1.0 + 0x1p-40);
    const double thi = __builtin_sqrt(t2_hi > 0.0 ? t2_hi : 0.0) * (1.0 + 0x1p-40);
    const double tlo = __builtin_sqrt(t2_lo > 0.0 ? t2_lo : 0.0) * (1.0 - 0x1p-40);
    const double up = (thi + R) * (1.0 + 0x1p-40);
    if (up * up * (1.0 + 0x1p-40) <= L.eps2_lo)
        return 1;
    const double dn = (tlo - R) * (1.0 - 0x1p-40);
    if (dn > 0.0 && dn * dn * (1.0 - 0x1p-40) > L.eps2_hi)
        return 0;
    return 2;
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma16x16x32(u16x8 a, u16x8 b, f32x4 c)
{
    if constexpr (PREC == 1)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                        __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                       __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}


// One wave per source point; 64 Philox calls (256 slots, 16 tiles) at a time.
// LDS per wave: the source row (KS*32 16-bit values) and 256 partner indices.
// kKB: K-steps of 32 whose partner fragments are in flight together.
template <int PREC, int kKB>
__global__ __launch_bounds__(256) void k_lowp_pass_a(Inst I, LowpArgs L, int KS)
{
    extern __shared__ uint16_t lds16[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int row_elems = KS * 32;
    uint16_t *xi_s = lds16 + (size_t)wib * (row_elems + 512);
    uint32_t *j_s = reinterpret_cast<uint32_t *>(xi_s + row_elems);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const int p = lane & 15;        // partner column of this lane
    const int kg = lane >> 4;       // k-group of this lane within a K-step
    uint32_t acc_self = 0, acc_acc = 0;

    for (uint64_t i = wave; i < I.n; i += nw) {  // wave-uniform
        // stage v_i (zero padded to KS*32) in LDS
        const uint16_t *vi = L.Xlp + i * L.ld_lp;
        for (int k = lane; k < row_elems; k += kWave)
            xi_s[k] = (k < I.d) ? vi[k] : (uint16_t)0;
        const double nvi = L.stats[4 * i + 0], ai = L.stats[4 * i + 1], ri = L.stats[4 * i + 2];
        uint32_t deg_i = 0;
        for (uint32_t c0 = 0; c0 < I.C; c0 += 64) {
            // partners of calls c0..c0+63
            const uint32_t c = c0 + (uint32_t)lane;
            const Words4 W = philox10(c, (uint32_t)i, I.key0, I.key1);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int w = 0; w < 4; ++w)
                j_s[4 * lane + w] = mod_exact(W.w[w], I.n, I.inv_n);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const uint32_t ncalls = min(64u, I.C - c0);
            const uint32_t ntiles = (ncalls + 3) / 4;
            for (uint32_t tile = 0; tile < ntiles; ++tile) {
                const uint32_t slot_in_batch = 16 * tile + p;       // 0..255
                const uint32_t t = 4 * c0 + slot_in_batch;            // sample index
                const bool valid = (t < I.m);
                const uint32_t jp = j_s[slot_in_batch];
                const uint32_t jr = valid ? jp : 0u;  // row 0 always exists
                const uint16_t *vj = L.Xlp + (uint64_t)jr * L.ld_lp + 8 * kg;
                const uint16_t *va = xi_s + 8 * kg;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                u16x8 b0[kKB], b1[kKB];
                auto fetch = [&](u16x8(&bb)[kKB], int s0) {
#pragma unroll
                    for (int q = 0; q < kKB; ++q) {
                        const int s = s0 + q;
                        const int k0 = 32 * s + 8 * kg;
                        u16x8 b = (u16x8){0, 0, 0, 0, 0, 0, 0, 0};
                        if (s < KS && k0 < I.d) {
                            b = *reinterpret_cast<const u16x8 *>(vj + 32 * s);
                            if (k0 + 8 > I.d) {
#pragma unroll
                                for (int e = 0; e < 8; ++e)
                                    if (k0 + e >= I.d)
                                        b[e] = 0;
                            }
                        }
                        bb[q] = b;
                    }
                };
                auto compute = [&](const u16x8(&bb)[kKB], int s0) {
#pragma unroll
                    for (int q = 0; q < kKB; ++q) {
                        const int s = s0 + q;
                        if (s < KS) {
                            const u16x8 a = *reinterpret_cast<const u16x8 *>(va + 32 * s);
                            acc = mfma16x16x32<PREC>(a, bb[q], acc);
                        }
                    }
                };
                // two register buffers of kKB fragments, alternated with
                // compile-time indices: one is in flight while the other is used
                fetch(b0, 0);
                for (int s0 = 0; s0 < KS; s0 += 2 * kKB) {
                    if (s0 + kKB < KS)
                        fetch(b1, s0 + kKB);
                    compute(b0, s0);
                    if (s0 + 2 * kKB < KS)
                        fetch(b0, s0 + 2 * kKB);
                    if (s0 + kKB < KS)
                        compute(b1, s0 + kKB);
                }
                // every row of A is v_i, so any row of column p is v_i . v_{j_p}
                int dec = 0;
                if (lane < 16 && valid) {
                    if (jp == (uint32_t)i) {
                        acc_self += 1;
                    } else {
                        const double nvj = L.stats[4 * (uint64_t)jp + 0];
                        const double aj = L.stats[4 * (uint64_t)jp + 1];
                        const double rj = L.stats[4 * (uint64_t)jp + 2];
                        dec = decide(L, acc[0], nvi, ai, ri, nvj, aj, rj);
                    }
                }
                if (dec == 1) {
                    if (!I.out_deg)
                        atomicAdd(I.deg + jp, 1u);
                    acc_acc += 1;
                    const uint64_t g = i * (uint64_t)I.C + (t >> 2);
                    atomicOr(I.mask + (g >> 3), 1u << (4 * (g & 7) + (t & 3)));
                }
                const uint64_t acc_ballot = __ballot(dec == 1);
                deg_i += __popcll(acc_ballot);
                const uint64_t rq = __ballot(dec == 2);
                if (rq) {
                    unsigned long long base = 0;
                    if (lane == 0)
                        base = atomicAdd(I.cnt + kCntQueue, (unsigned long long)__popcll(rq));
                    base = __shfl(base, 0);
                    if (dec == 2) {
                        const uint64_t pos = base + __popcll(rq & ((1ull << lane) - 1));
                        if (pos < L.qcap)
                            L.queue[pos] = i * (uint64_t)I.m + t;
                        else
                            atomicOr(I.cnt + kCntOverflow, 1ull);
                    }
                }
            }
        }
        if (lane == 0 && deg_i)
            atomicAdd(I.deg + i, deg_i);
        __builtin_amdgcn_wave_barrier();
    }
    const int slots[2] = {kCntSelf, kCntAccepted};
    const uint32_t v[2] = {acc_self, acc_acc};
    block_count_add<2>(I.cnt, slots, v);
}

// Re-decides every queued slot with the defining binary64 sum. A wavefront
// takes 64 queued slots at a time, lane l owning slot l's sum. The squared
// binary64 differences are independent of each other, so they are computed
// kRecheckK coordinates at a time with coalesced row loads (two pairs per
// step, one per half-wave) and parked in LDS; then each lane adds its own
// pair's terms in coordinate order, which keeps the defining sequence of
// roundings.
constexpr int kRecheckK = 32;               // coordinates per LDS chunk
constexpr int kRecheckStride = kWave + 1;   // doubles per LDS row (padding)
constexpr int kRecheckWaves = 4;

__global__ __launch_bounds__(kWave * kRecheckWaves) void k_lowp_recheck(Inst I, LowpArgs L)
{
#pragma clang fp contract(off)
    __shared__ double terms[kRecheckWaves][kRecheckK * kRecheckStride];
    double *T = terms[threadIdx.x / kWave];
    const int lane = lane_id();
    const int half = lane >> 5;
    const int kl = lane & 31;
    const unsigned long long q = min((unsigned long long)I.cnt[kCntQueue],
                                     (unsigned long long)L.qcap);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * blockDim.x / kWave;
    const int d = I.d;
    uint32_t acc_n = 0;
    for (uint64_t e0 = wave * kWave; e0 < q; e0 += waves * kWave) {  // wave-uniform
        const uint64_t e = e0 + (uint64_t)lane;
        const bool live = e < q;
        uint32_t i = 0, j = 0, t = 0;
        if (live) {
            const uint64_t u = L.queue[e];
            const uint64_t ii = u / I.m;
            t = (uint32_t)(u - ii * I.m);
            i = (uint32_t)ii;
            const Words4 W = philox10(t >> 2, i, I.key0, I.key1);
            j = mod_exact(W.w[t & 3], I.n, I.inv_n);
        }
        const int npairs = (int)min((uint64_t)kWave, q - e0);
        double acc = 0.0;
        for (int k0 = 0; k0 < d; k0 += kRecheckK) {
            const int k = k0 + kl;
            for (int pp = 0; pp < npairs; pp += 2) {  // wave-uniform
                const uint32_t i0 = (uint32_t)__builtin_amdgcn_readlane((int)i, pp);
                const uint32_t j0 = (uint32_t)__builtin_amdgcn_readlane((int)j, pp);
                const int p1 = pp + 1 < npairs ? pp + 1 : pp;
                const uint32_t i1 = (uint32_t)__builtin_amdgcn_readlane((int)i, p1);
                const uint32_t j1 = (uint32_t)__builtin_amdgcn_readlane((int)j, p1);
                const uint32_t ip = half ? i1 : i0;
                const uint32_t jp = half ? j1 : j0;
                double sq = 0.0;
                if (k < d) {
                    const double delta = (double)I.X[(uint64_t)ip * I.ld + k] -
                                         (double)I.X[(uint64_t)jp * I.ld + k];
                    sq = delta * delta;
                }
                T[kl * kRecheckStride + pp + half] = sq;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int kn = min(kRecheckK, d - k0);
            if (live) {
                for (int c = 0; c < kn; ++c)
                    acc = acc + T[c * kRecheckStride + lane];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (live && acc <= I.eps2) {
            atomicAdd(I.deg + i, 1u);
            if (!I.out_deg)
                atomicAdd(I.deg + j, 1u);
            const uint64_t g = (uint64_t)i * (uint64_t)I.C + (t >> 2);
            atomicOr(I.mask + (g >> 3), 1u << (4 * (g & 7) + (t & 3)));
            acc_n += 1;
        }
    }
    const int slots[1] = {kCntAccepted};
    const uint32_t v[1] = {acc_n};
    block_count_add<1>(I.cnt, slots, v);
}

__global__ void k_lowp_count_rechecked(unsigned long long *cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        cnt[kCntRechecked] = cnt[kCntQueue];
}

hipError_t launch_lowp(const Inst &I, const LowpArgs &L, int prec, hipStream_t st, int waves_req,
                       int ksteps)
{
    if (I.n == 0 || I.m == 0)
        return hipSuccess;
    const int KS = (I.d + 31) / 32;
    const size_t lds_per_wave = ((size_t)KS * 32 + 512) * sizeof(uint16_t);
    int waves = 4;
    while (waves > 1 && lds_per_wave * waves > 65536)
        waves >>= 1;
    if (waves_req != 0) {
        if (waves_req != 1 && waves_req != 2 && waves_req != 4)
            return hipErrorInvalidValue;
        waves = waves_req;
    }
    if (ksteps == 0)
        ksteps = 8;
    if (ksteps != 4 && ksteps != 8 && ksteps != 16)
        return hipErrorInvalidValue;
    if (lds_per_wave * waves > 65536)
        return hipErrorInvalidValue;
    const uint64_t sb = ((uint64_t)I.n + 3) / 4;
    const unsigned stat_blocks = (unsigned)(sb < 4096 ? sb : 4096);
    if (prec == 1)
        hipLaunchKernelGGL(k_rowstats<1>, dim3(stat_blocks), dim3(256), 0, st, I, L);
    else
        hipLaunchKernelGGL(k_rowstats<2>, dim3(stat_blocks), dim3(256), 0, st, I, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_rowstats_summary, dim3(1), dim3(kSummaryThreads), 0, st, I, L);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    const uint64_t nb = ((uint64_t)I.n + waves - 1) / waves;
    const unsigned blocks = (unsigned)(nb < 8192 ? nb : 8192);
    const size_t lds = lds_per_wave * waves;
#define SNG_LOWP_LAUNCH(P, KB)                                                                 \
    hipLaunchKernelGGL((k_lowp_pass_a<P, KB>), dim3(blocks), dim3(64 * waves), lds, st, I, L, KS)
    if (prec == 1) {
        if (ksteps == 4) SNG_LOWP_LAUNCH(1, 4);
        else if (ksteps == 8) SNG_LOWP_LAUNCH(1, 8);
        else SNG_LOWP_LAUNCH(1, 16);
    } else {
        if (ksteps == 4) SNG_LOWP_LAUNCH(2, 4);
        else if (ksteps == 8) SNG_LOWP_LAUNCH(2, 8);
        else SNG_LOWP_LAUNCH(2, 16);
    }
#undef SNG_LOWP_LAUNCH
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_lowp_recheck, dim3(1024), dim3(kWave * kRecheckWaves), 0, st, I, L);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_lowp_count_rechecked, dim3(1), dim3(64), 0, st, I.cnt);
    return hipGetLastError();
}

}  // namespace sng
