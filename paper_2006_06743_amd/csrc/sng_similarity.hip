// Similarity queries other than the distance (the method only needs a yes/no
// similarity query per sampled pair, Section 1): an edge when the dot product
// or the cosine of the pair is at least tau. The sampled-distance pass runs
// unchanged and decides each slot from its binary32 squared distance through
// the per-pair band of SimQuery (polarisation), with the binary64 definition
// inside the band; this file holds the per-row statistics that band needs
// and the host-side band constants.
#include <math.h>

#include "sng_internal.hpp"

namespace sng {

namespace {

// Rows whose squared norm lies outside [2^-100, 2^100] (zero rows included)
// keep NaN statistics, so every pair touching them goes to binary64: there
// the binary32 norms could underflow or overflow.
constexpr double kNormMin = 0x1p-100, kNormMax = 0x1p100;

// G lanes per row; lane q sums coordinates q, q+G, ... in binary64 and the
// group adds the partial sums (any order: the band allows for it).
template <int G>
__global__ __launch_bounds__(256) void k_row_norms(const float *__restrict__ X, int64_t ld,
                                                   uint32_t n, int d, float2 *__restrict__ nrm)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const int q = (int)(threadIdx.x & (G - 1));
    const uint64_t rows = (uint64_t)n * G;
    // whole groups stay together: rows * G and the stride are multiples of G
    for (uint64_t r = tid; r < rows; r += stride) {
        const uint64_t i = r / G;
        const float *x = X + (int64_t)i * ld;
        double s = 0.0;
        for (int k = q; k < d; k += G) {
            const double v = (double)x[k];
            s += v * v;
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1)
            s += __shfl_xor(s, o, G);
        if (q == 0) {
            float2 v;
            if (s >= kNormMin && s <= kNormMax) {
                v.x = (float)s;
                v.y = (float)__builtin_sqrt(s);
            } else {
                v.x = v.y = __builtin_nanf("");
            }
            nrm[i] = v;
        }
    }
}

float round_up_f32(double v)
{
    float f = (float)v;
    if ((double)f < v)
        f = nextafterf(f, INFINITY);
    return f;
}

}  // namespace

void set_similarity(Inst &I, int32_t kind, double tau, float2 *nrm)
{
    // a = gamma_{d+2} of binary32, as in the distance band; k = 2a + 2^-19
    // covers the binary64 definition, the binary32 norms and the binary32
    // arithmetic of the threshold (see SimQuery)
    const double u32 = 0x1p-24;
    const double ka = (double)I.d + 2.0;
    double k = INFINITY;
    if (ka * u32 < 0.5)
        k = (2.0 * (ka * u32 / (1.0 - ka * u32)) + 0x1p-19) * (1.0 + 0x1p-20);
    I.sim.nrm = nrm;
    I.sim.kind = kind;
    I.sim.t = (float)tau;
    I.sim.k = round_up_f32(k);
    I.sim.beta = round_up_f32(2.0 * (2.0 * I.d + 2.0) * 0x1p-126);
    I.sim.tau = tau;
    I.band = k;
    // the distance band is never used by a similarity instance
    I.lo = -1.0f;
    I.hi = INFINITY;
}

hipError_t launch_row_norms(const Inst &I, float2 *nrm, hipStream_t st)
{
    if (I.n == 0)
        return hipSuccess;
    int g = 1;
    while (g < I.d && g < 64)
        g <<= 1;
    const uint64_t threads = (uint64_t)I.n * g;
    uint64_t blocks = (threads + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
#define SNG_NORMS(GG)                                                                          \
    case GG:                                                                                   \
        hipLaunchKernelGGL((k_row_norms<GG>), dim3((unsigned)blocks), dim3(256), 0, st, I.X,   \
                           I.ld, I.n, I.d, nrm);                                               \
        break;
    switch (g) {
        SNG_NORMS(1)
        SNG_NORMS(2)
        SNG_NORMS(4)
        SNG_NORMS(8)
        SNG_NORMS(16)
        SNG_NORMS(32)
        SNG_NORMS(64)
    }
#undef SNG_NORMS
    return hipGetLastError();
}

}  // namespace sng
