// Similarity queries other than the distance (the method only needs a yes/no
// similarity query per sampled pair, Section 1): an edge when the dot product
// or the cosine of the pair is at least tau. The sampled-distance kernels
// filter in binary32 and the binary64 definition decides within the filter's
// error bound (SimQuery). This file holds what runs before the pass and the
// host-side constants:
//   cosine       a copy of the rows scaled to unit length, on which
//                cos >= tau is |u - v|^2 <= 2 - 2 tau, and its band;
//   dot product  the constants of its filter on P = sum a_k b_k and
//                Q = sum |a_k b_k| (the pass needs no per-row data).
#include <math.h>

#include "sng_internal.hpp"

namespace sng {

namespace {

// Rows whose squared norm lies outside [2^-100, 2^100] (zero rows included)
// get a NaN copy, so every pair touching them goes to binary64: there the
// scaled binary32 values could underflow or overflow.
constexpr double kNormMin = 0x1p-100, kNormMax = 0x1p100;

// Squared norm of row i by the G lanes of its group: lane q sums coordinates
// q, q+G, ... in binary64 and the group adds the partial sums (any order: the
// bands allow for it). Every lane of the group gets the total.
template <int G>
__device__ __forceinline__ double row_sq(const float *__restrict__ x, int d, int q)
{
    double s = 0.0;
    for (int k = q; k < d; k += G) {
        const double v = (double)x[k];
        s += v * v;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
        s += __shfl_xor(s, o, G);
    return s;
}

// Grid-stride over (row, lane) pairs; rows * G and the stride are multiples
// of G, so the G lanes of a row stay together.
// U[i][k] = fl32(x_ik / |x_i|) for k < d, 0 up to ldu (NaN row when the
// squared norm is out of range).
template <int G>
__global__ __launch_bounds__(256) void k_unit_rows(const float *__restrict__ X, int64_t ld,
                                                   uint32_t n, int d, float *__restrict__ U,
                                                   int64_t ldu)
{
    const int q = (int)(threadIdx.x & (G - 1));
    const uint64_t rows = (uint64_t)n * G, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += stride) {
        const uint64_t i = r / G;
        const float *x = X + (int64_t)i * ld;
        const double s = row_sq<G>(x, d, q);
        const bool ok = s >= kNormMin && s <= kNormMax;
        const double inv = ok ? 1.0 / __builtin_sqrt(s) : 0.0;
        float *u = U + (int64_t)i * ldu;
        for (int k = q; k < (int)ldu; k += G)
            u[k] = k >= d ? 0.0f : (ok ? (float)((double)x[k] * inv) : __builtin_nanf(""));
    }
}

int lanes_for(int d)
{
    int g = 1;
    while (g < d && g < 64)
        g <<= 1;
    return g;
}

template <template <int> class K, class... Args>
hipError_t launch_rows(uint32_t n, int d, hipStream_t st, Args... args)
{
    if (n == 0)
        return hipSuccess;
    const int g = lanes_for(d);
    uint64_t blocks = ((uint64_t)n * g + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    const dim3 grid((unsigned)blocks), block(256);
    switch (g) {
    case 1: hipLaunchKernelGGL(K<1>::fn, grid, block, 0, st, args...); break;
    case 2: hipLaunchKernelGGL(K<2>::fn, grid, block, 0, st, args...); break;
    case 4: hipLaunchKernelGGL(K<4>::fn, grid, block, 0, st, args...); break;
    case 8: hipLaunchKernelGGL(K<8>::fn, grid, block, 0, st, args...); break;
    case 16: hipLaunchKernelGGL(K<16>::fn, grid, block, 0, st, args...); break;
    case 32: hipLaunchKernelGGL(K<32>::fn, grid, block, 0, st, args...); break;
    default: hipLaunchKernelGGL(K<64>::fn, grid, block, 0, st, args...); break;
    }
    return hipGetLastError();
}

template <int G>
struct UnitRows {
    static constexpr auto fn = k_unit_rows<G>;
};

float round_up_f32(double v)
{
    float f = (float)v;
    if ((double)f < v)
        f = nextafterf(f, INFINITY);
    return f;
}

float round_down_f32(double v)
{
    float f = (float)v;
    if ((double)f > v)
        f = nextafterf(f, -INFINITY);
    return f;
}

}  // namespace

int64_t unit_copy_ld(int32_t d)
{
    return ((int64_t)d + 3) & ~(int64_t)3;
}

void set_similarity(Inst &I, int32_t kind, double tau, float *unit)
{
    const double u32 = 0x1p-24, u64 = 0x1p-53;
    const double d = (double)I.d;
    const double beta = (2.0 * d + 2.0) * 0x1p-126;  // flushed binary32 subnormals
    I.sim.X0 = I.X;
    I.sim.ld0 = I.ld;
    I.sim.kind = kind;
    I.sim.tau = tau;
    if (kind == kSimCos) {
        // On the unit copy u, v of rows a, b: each coordinate is within
        // delta = 2^-24 (1 + 2^-20) of a_k/|a| relative (binary64 norm and
        // quotient, one binary32 rounding), so | |u - v|^2 - (2 - 2 cos) | <=
        // 8.1 delta (unit-length distances are at most 2); the binary32 F is
        // within 4.02 a + beta of |u - v|^2 (a = gamma_{d+2} of binary32, as
        // for the distance); the binary64 cosine within (2d + 8) 2^-53 of the
        // exact one. F <= 2 - 2 tau - H then forces the definition to accept
        // and F > 2 - 2 tau + H to reject.
        const double ka = d + 2.0;
        const double a = ka * u32 < 0.5 ? ka * u32 / (1.0 - ka * u32) : INFINITY;
        const double delta = u32 * (1.0 + 0x1p-20);
        const double e64 = (2.0 * d + 8.0) * u64;
        const double H = (4.02 * a + 8.1 * delta + beta + 2.0 * e64 + 0x1p-100) * (1.0 + 0x1p-20);
        const double c = 2.0 - 2.0 * tau;
        I.lo = isinf(H) ? -1.0f : round_down_f32(c - H);
        I.hi = isinf(H) ? INFINITY : round_up_f32(c + H);
        I.band = H;
        I.X = unit;
        I.ld = unit_copy_ld(I.d);
    } else {
        // Dot product: |P - <a,b>| <= gamma_d S + beta and |definition -
        // <a,b>| <= gamma_d(binary64) S, S = sum |a_k b_k| <= (Q + beta) /
        // (1 - gamma_d). k covers both relative terms with 2^-20 to spare
        // (more than the binary32 rounding of k Q, t + H and t - H); c covers
        // the subnormal terms and the rounding of tau to binary32 (2^-24 |t|)
        // and of the threshold sums (another 2^-24 |t| each side).
        const double gd = d * u32 < 0.5 ? d * u32 / (1.0 - d * u32) : INFINITY;
        const double g64 = 2.0 * (d + 2.0) * u64;
        const double k = isinf(gd) ? INFINITY : (gd + g64) / (1.0 - gd) * (1.0 + 0x1p-20);
        I.sim.t = (float)tau;
        I.sim.k = round_up_f32(k);
        I.sim.c = round_up_f32(3.0 * beta + 3.0 * u32 * fabs((double)I.sim.t));
        I.band = k;
        I.lo = -1.0f;  // the distance band is not used
        I.hi = INFINITY;
    }
}

hipError_t launch_similarity_rows(const Inst &I, float *unit, hipStream_t st)
{
    if (I.sim.kind != kSimCos)
        return hipSuccess;  // the dot-product filter needs no per-row data
    return launch_rows<UnitRows>(I.n, I.d, st, I.sim.X0, I.sim.ld0, I.n, I.d, unit,
                                 unit_copy_ld(I.d));
}

}  // namespace sng
