// Device building blocks of the SNG-DBSCAN kernels (gfx950, wave64).
//
// Everything here runs on the GPU; the host side only fills the Inst
// descriptor. Nothing is shared with the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sng {

constexpr int kWave = 64;
constexpr int32_t kNoCore = 0x7FFFFFFF;  // "no core neighbour yet" in the label array

// Counter slots in the workspace header (u64 each).
enum Counter : int {
    kCntSlots = 0,
    kCntSelf = 1,
    kCntAccepted = 2,
    kCntRechecked = 3,
    kCntCore = 4,
    kCntClusters = 5,
    kCntNoise = 6,
    kCntOverflow = 7,
    kCntQueue = 8,
    kCntNum = 16
};
// Header words of the mixed form's filter (doubles unless noted), cleared
// with the counters: its error constants, then max and sum of the rows'
// rounding radii and norms.
enum {
    kFltGamma = 17,
    kFltGammaNorm = 18,
    kFltScale2 = 19,
    kFltEps2 = 20,
    kFltRMax = 21,
    kFltAMax = 22,
    kFltRSum = 23,
    kFltASum = 24,
    kFltRows = 25,  // u64
    kFltEnd = 26
};

// Similarity queries other than the distance: an edge when the dot product
// (kSimDot) or the cosine (kSimCos) of the pair is at least tau; binary64 in
// coordinate order decides, as for the distance. The binary32 pass filters
// and the definition decides inside the filter's error bound:
//
// Cosine: the pass runs the distance kernels on a copy of the rows scaled to
// unit length, where |u - v|^2 = 2 - 2 cos, so cos >= tau is the distance
// test against the constant 2 - 2 tau; its band (the instance's lo, hi, set
// on the host) also covers the rounding of the scaled copy.
//
// Dot product: the pass forms P = sum a_k b_k and Q = sum |a_k b_k| in
// binary32 (any order, fused or not). |P - <a,b>| <= gamma_d (in binary32)
// times sum |a_k b_k| <= gamma_d Q / (1 - gamma_d), plus flushed subnormals,
// and the binary64 definition is within gamma_d (binary64) of the same sum;
// so P above t + H surely reaches tau and P below t - H surely does not,
// with H = k Q + c (k and c set on the host, c also covering the binary32
// rounding of tau and of this arithmetic).
enum : int32_t { kSimNone = 0, kSimDot = 1, kSimCos = 2 };

struct SimQuery {
    const float *X0;    // the caller's rows, for the binary64 definition
    int64_t ld0;        // their stride in floats
    int32_t kind;       // kSimNone: the distance query (the other fields unused)
    float t;            // dot product: fl32(tau)
    float k;            // dot product: relative half-width (times Q)
    float c;            // dot product: absolute half-width
    double tau;         // the threshold of the binary64 definition

    // Dot-product decision from P and Q: 1 surely an edge, 0 surely not,
    // -1 undecided (NaN or infinite operands included).
    __device__ __forceinline__ int band_dot(float P, float Q) const
    {
        const float H = k * Q + c;
        if (P > t + H)
            return 1;
        if (P < t - H)
            return 0;
        return -1;
    }
};

// One clustering instance as the kernels see it.
struct Inst {
    const float *X;         // row-major, element (i,k) at X[i*ld + k]
    int64_t ld;             // row stride in floats
    uint32_t n;             // points
    int32_t d;              // dimension
    uint32_t m;             // samples per point
    uint32_t C;             // Philox calls per point = ceil(m/4)
    uint32_t key0, key1;    // Philox key = seed
    double inv_n;           // fl64(1/n), for the exact remainder
    float inv_nf;           // fl32(fl64(1/n)) when 1024 <= n <= 2^30, else 0
    double inv_C;           // fl64(1/C)
    float lo, hi;           // binary32 band: F <= lo accept, F > hi reject
    double eps2;            // fl64(eps*eps), the binary64 threshold
    uint64_t calls;         // n*C
    uint64_t chunk0;        // first global 64-call chunk of this instance
    uint64_t chunks;        // chunks of this instance
    uint32_t *deg;          // [n] degrees (symmetrised, or out-degrees if out_deg)
    uint32_t *mask;         // accept bits, 32 per word = 8 calls; indexed by global call
    uint8_t *core;          // [n]
    int32_t *labels;        // [n] union-find parents / border candidates / labels
    unsigned long long *cnt;  // counters (kCntNum)
    int32_t min_pts;
    int32_t out_deg;        // 1: a point's degree counts only its own accepted samples
    double band;              // relative half-width of the binary32 band (reported)
    SimQuery sim;           // kind kSimNone: the distance against eps2
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11, Sec. 3.2) for the counter (c, i, 0, 0).
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w[4];
};

// a ^ b ^ c in one instruction: gfx950's three-input bit operation with the
// odd-parity truth table 0x96 (symmetric, so the operand order is free).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words4 philox10(uint32_t c, uint32_t i, uint32_t key0, uint32_t key1)
{
    uint32_t x0 = c, x1 = i, x2 = 0u, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p = (uint64_t)0xD2511F53u * x0;  // multiplier 0
        const uint64_t q = (uint64_t)0xCD9E8D57u * x2;  // multiplier 1
        const uint32_t y0 = xor3((uint32_t)(q >> 32), x1, key0);
        const uint32_t y2 = xor3((uint32_t)(p >> 32), x3, key1);
        x1 = (uint32_t)q;
        x3 = (uint32_t)p;
        x0 = y0;
        x2 = y2;
        key0 += 0x9E3779B9u;  // Weyl increments: golden ratio, sqrt(3)-1
        key1 += 0xBB67AE85u;
    }
    Words4 o;
    o.w[0] = x0;
    o.w[1] = x1;
    o.w[2] = x2;
    o.w[3] = x3;
    return o;
}

// Exact w mod n for w < 2^32, 1 <= n < 2^31. The binary64 quotient estimate
// is within 2^-20 of w/n, so the truncated quotient is off by at most one and
// a single correction step lands in [0, n).
__device__ __forceinline__ uint32_t mod_exact(uint32_t w, uint32_t n, double inv_n)
{
    const uint32_t q = (uint32_t)((double)w * inv_n);
    int64_t r = (int64_t)w - (int64_t)q * (int64_t)n;
    r += (r < 0) ? (int64_t)n : 0;
    r -= (r >= (int64_t)n) ? (int64_t)n : 0;
    return (uint32_t)r;
}

// Exact w mod n for 1024 <= n <= 2^30 from a binary32 quotient estimate.
// fl32(w), inv = fl32(fl64(1/n)) and their rounded product each carry a
// relative error below 2^-24 (1 + 2^-28), so the estimate is within
// (w/n) * 3.0001 * 2^-24 < 2^22 * 3.0001 * 2^-24 < 1 of w/n, and its
// truncation q is one of floor(w/n) - 1, floor(w/n), floor(w/n) + 1. Then
// w - q n lies in [-n, 2n), which 32-bit wrap-around holds exactly as n <=
// 2^30, and of r, r + n and r - n exactly one lies in [0, n): the others are
// at least n, or wrap to at least 2^32 - 2n >= 2^31. Their unsigned minimum
// is the remainder.
__device__ __forceinline__ uint32_t mod_f32(uint32_t w, uint32_t n, float inv)
{
    const uint32_t q = (uint32_t)((float)w * inv);
    const uint32_t r = w - q * n;
    return min(min(r, r + n), r - n);
}

// The same for n < 2^24: the quotient estimate is below 2^32 / 1024 = 2^22,
// so q * n is a 24-bit multiply (full rate) whose low 32 bits are all the
// remainder needs.
__device__ __forceinline__ uint32_t mod_f32_n24(uint32_t w, uint32_t n, float inv)
{
    const uint32_t q = (uint32_t)((float)w * inv);
    const uint32_t r = w - __umul24(q, n);
    return min(min(r, r + n), r - n);
}

// w mod n for 4096 <= n <= 2^23 from a quotient estimate that never exceeds
// w/n. inv is (1/n)(1 - 2^-21) rounded down to binary32, so it lies within
// 2^-23 (relative) below that value; fl32(w) and the rounded product add a
// relative error below 2^-24 each. The estimate p then satisfies
// (w/n)(1 - 3 * 2^-22) < p < w/n, and as w/n < 2^32 / 2^12 = 2^20 it is
// less than 0.75 below w/n: its truncation q is floor(w/n) or one less.
// So r = w - q n lies in [0, 2n), and min(r, r - n) is the remainder (r - n
// wraps above r when r < n). q < 2^20 and -n >= -2^23 are signed 24-bit
// operands, so q n and the subtraction are one 24-bit multiply-add.
__device__ __forceinline__ uint32_t mod_f32_floor(uint32_t w, uint32_t n, float inv)
{
    const int32_t q = (int32_t)(uint32_t)((float)w * inv);
    const uint32_t r = (uint32_t)((int32_t)w + __mul24(q, -(int32_t)n));
    return min(r, r - n);
}

// The four partners of one Philox call: its words mod n. The branch is
// uniform (one instance per wavefront), so only one side runs.
__device__ __forceinline__ void partners4(const Inst &I, const Words4 &W, uint32_t j[4])
{
    if (I.inv_nf != 0.0f) {
#pragma unroll
        for (int w = 0; w < 4; ++w)
            j[w] = mod_f32(W.w[w], I.n, I.inv_nf);
    } else {
#pragma unroll
        for (int w = 0; w < 4; ++w)
            j[w] = mod_exact(W.w[w], I.n, I.inv_n);
    }
}

// Exact floor division a / b for a < 2^40 and 1 <= b < 2^32: the binary64
// estimate of a / b is within one of the quotient, then corrected.
__device__ __forceinline__ uint64_t div_exact64(uint64_t a, uint32_t b, double inv_b)
{
    uint64_t q = (uint64_t)((double)a * inv_b);
    const int64_t r = (int64_t)a - (int64_t)(q * (uint64_t)b);
    if (r < 0)
        q -= 1;
    else if (r >= (int64_t)b)
        q += 1;
    return q;
}

// Space for `n` items in a workgroup-shared list: one LDS atomic per
// wavefront (lanes may ask for zero). Returns this lane's first index.
__device__ __forceinline__ uint32_t list_reserve(uint32_t n, uint32_t *count)
{
    uint32_t incl = n;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint32_t u = __shfl_up(incl, s);
        if ((int)__lane_id() >= s)
            incl += u;
    }
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    uint32_t base = 0;
    if (__lane_id() == 63 && total)
        base = atomicAdd(count, total);
    base = (uint32_t)__shfl((int)base, 63);
    return base + incl - n;
}

// floor(a / C) for a < 2^31 by multiply and shift (Granlund and Montgomery,
// PLDI 1994, Thm 4.2 with N = 31): with l = ceil(log2 C) and
// m = ceil(2^(31+l) / C) < 2^32, floor(a / C) = floor(a * m / 2^(31+l)).
struct DivMagic {
    uint32_t m;
    uint32_t shift;  // 31 + l
};
__device__ __forceinline__ uint32_t div_magic(uint32_t a, DivMagic dm)
{
    return (uint32_t)(((uint64_t)a * dm.m) >> dm.shift);
}

// Raw buffer access: 32-bit byte offsets from a base address; offsets at or
// past `bytes` read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bld1(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ float4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}

// Logical block of a grid whose size is a multiple of 8: workgroup b is
// dispatched to XCD b mod 8, so XCD x gets the logical blocks
// [x * nb / 8, (x + 1) * nb / 8), a contiguous eighth of the work, taken in
// order. Any dispatch order gives the same results; this one keeps each
// XCD's data in its own L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    return (b % 8u) * (nb / 8u) + b / 8u;
}

// Exact floor division a / b for a, b < 2^32 (same argument as mod_exact).
__device__ __forceinline__ uint32_t div_exact(uint32_t a, uint32_t b, double inv_b)
{
    uint32_t q = (uint32_t)((double)a * inv_b);
    int64_t r = (int64_t)a - (int64_t)q * (int64_t)b;
    if (r < 0)
        q -= 1;
    else if (r >= (int64_t)b)
        q += 1;
    return q;
}

// ---------------------------------------------------------------------------
// Cross-lane helpers within a group of G consecutive lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Value of `v` held by lane `o` of this lane's group of G lanes. `o` is a
// compile-time constant after unrolling for G <= 4.
template <int G>
__device__ __forceinline__ uint32_t group_bcast(uint32_t v, int o)
{
    if constexpr (G == 1) {
        return v;
    } else if constexpr (G == 2) {
        // quad_perm [o, o, 2+o, 2+o]
        switch (o) {
        case 0: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xA0, 0xF, 0xF, false);
        default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xF5, 0xF, 0xF, false);
        }
    } else if constexpr (G == 4) {
        switch (o) {
        case 0: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x00, 0xF, 0xF, false);
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x55, 0xF, 0xF, false);
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xAA, 0xF, 0xF, false);
        default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xFF, 0xF, 0xF, false);
        }
    } else if constexpr (G == 64) {
        return (uint32_t)__builtin_amdgcn_readlane((int)v, o);
    } else {
        const int src = (lane_id() & ~(G - 1)) + o;
        return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
    }
}


template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float xor_f(float v, int mask)
{
    const int src = lane_id() ^ mask;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Sum over the G lanes of a group; every lane of the group receives the
// same bits (pairings are symmetric and float addition is commutative).
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (G >= 64)
        v += xor_f(v, 32);
    if constexpr (G >= 32)
        v += xor_f(v, 16);
    if constexpr (G >= 16)
        v += dpp_f<0x140>(v);  // row_mirror: lane l <-> 15-l within 16
    if constexpr (G >= 8)
        v += dpp_f<0x141>(v);  // row_half_mirror: lane l <-> 7-l within 8
    if constexpr (G >= 4)
        v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (G >= 2)
        v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
    return v;
}

// The group's first lane's value in every lane of the group: makes a value
// that a reduction left equal across the group uniform to the compiler.
template <int G>
__device__ __forceinline__ float group_all(float v)
{
    return __int_as_float((int)group_bcast<G>((uint32_t)__float_as_int(v), 0));
}

// OR of a value over 8 consecutive lanes (lanes 8k..8k+7); all receive it.
__device__ __forceinline__ uint32_t or8(uint32_t v)
{
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// Adds K per-thread tallies into cnt[slot[k]] with one atomic per block and
// counter (every thread of the block must call it; blockDim <= 1024).
template <int K>
__device__ __forceinline__ void block_count_add(unsigned long long *cnt, const int (&slot)[K],
                                                const uint32_t (&mine)[K])
{
    __shared__ unsigned long long part[K][16];
    const int w = threadIdx.x / kWave;
    unsigned long long s[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        s[k] = wave_sum_u64(mine[k]);
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            part[k][w] = s[k];
    }
    __syncthreads();
    if (threadIdx.x < K && cnt) {
        const int nw = (blockDim.x + kWave - 1) / kWave;
        unsigned long long tot = 0;
        for (int i = 0; i < nw; ++i)
            tot += part[threadIdx.x][i];
        if (tot)
            atomicAdd(cnt + slot[threadIdx.x], tot);
    }
}

// ---------------------------------------------------------------------------
// binary64 squared distance in the defining order: sequential over k,
// rounded to nearest-even at every step, never fused.
// ---------------------------------------------------------------------------
__device__ __noinline__ double sqdist_f64(const float *__restrict__ a, const float *__restrict__ b,
                                         int d)
{
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        const double delta = (double)a[k] - (double)b[k];
        const double sq = delta * delta;
        acc = acc + sq;
    }
    return acc;
}

// The binary64 definitions of the similarity queries: the dot product in
// coordinate order, and the cosine ip / (sqrt(|a|^2) * sqrt(|b|^2)) with each
// squared norm summed the same way (0 / 0 for a zero row: no edge).
__device__ __noinline__ int sim_accept_f64(const float *__restrict__ a,
                                           const float *__restrict__ b, int d, int kind,
                                           double tau)
{
#pragma clang fp contract(off)
    double ip = 0.0;
    for (int k = 0; k < d; ++k) {
        const double p = (double)a[k] * (double)b[k];
        ip = ip + p;
    }
    if (kind == kSimDot)
        return ip >= tau;
    double na = 0.0, nb = 0.0;
    for (int k = 0; k < d; ++k) {
        const double p = (double)a[k] * (double)a[k];
        na = na + p;
    }
    for (int k = 0; k < d; ++k) {
        const double p = (double)b[k] * (double)b[k];
        nb = nb + p;
    }
    const double den = __builtin_sqrt(na) * __builtin_sqrt(nb);
    return ip / den >= tau;
}

// ---------------------------------------------------------------------------
// Lock-free union-find on the label array. Parents always point to smaller
// indices, so the root of a component is its minimum member.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way (any written value is an ancestor,
// so concurrent finds and hooks stay consistent).
//
// The walk reads and writes the forest through the compute unit's own
// caches (workgroup-scope relaxed accesses), so it may see parent pointers
// that other XCDs have since lowered. That is safe for three reasons: a
// parent always has a smaller index than its child, so any walk ends; every
// pointer ever stored joins two points of one component, so a stale root
// still names the right component, and a stale halving store still writes an
// ancestor; and the compare-and-swap that hooks a root acts at device scope
// on the current value, so it fails on an entry that has stopped being a root
// and the retry starts from the fresh value it returns (hooking under a stale
// root is harmless: that point is in the same component and has a smaller
// index). The forest is fully written back when the kernel ends. Device-scope
// reads instead go past the XCD's L2 on every step of every walk, which is
// what the hooks of dense clusters spend their time on.
__device__ __forceinline__ int32_t uf_ld(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void uf_st(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t uf_find(int32_t *P, int32_t x)
{
    int32_t p = uf_ld(P + x);
    while (p != x) {
        const int32_t gp = uf_ld(P + p);
        if (gp == p)
            return p;
        uf_st(P + x, gp);
        x = gp;
        p = uf_ld(P + x);
    }
    return x;
}

// Root of x without writing anything. Used once the forest is final, when
// each entry is rewritten only by its own thread: a walk that halved paths
// could store an intermediate ancestor into an entry after that entry's own
// thread had stored the root.
__device__ __forceinline__ int32_t uf_root(const int32_t *P, int32_t x)
{
    int32_t p = ld_relaxed(P + x);
    while (p != x) {
        x = p;
        p = ld_relaxed(P + x);
    }
    return x;
}

// Join the components of a and b: the larger root is hooked under the
// smaller one by compare-and-swap, retrying from the new roots on conflict.
__device__ __forceinline__ void uf_unite(int32_t *P, int32_t a, int32_t b)
{
    int32_t ra = uf_find(P, a), rb = uf_find(P, b);
    while (ra != rb) {
        if (ra > rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        const int32_t old = atomicCAS(P + rb, rb, ra);
        if (old == rb)
            return;
        rb = uf_find(P, old);
        ra = uf_find(P, ra);
    }
}

}  // namespace sng
