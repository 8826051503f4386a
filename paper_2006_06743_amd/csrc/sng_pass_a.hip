// Sampled-distance pass of SNG-DBSCAN (Algorithm 1, graph construction):
// every sample slot (i, t) draws its partner j from Philox, gathers row j,
// decides |x_i - x_j| <= eps and, on acceptance, adds one to the degree of
// both endpoints. Edges are never stored; the accept decision of each slot
// is kept as one bit so that the hook pass can regenerate exactly the
// accepted pairs without a second gather of X.
//
// Work decomposition (wave64): a wavefront owns chunks of 64 consecutive
// Philox calls (one call = four slots of one source point). Lane l computes
// call l of the chunk. Lanes are grouped G at a time; a group walks the 4G
// slots of its own G calls one after another, the G lanes splitting the
// coordinates of the pair, so each gathered row is read by one coalesced
// access of G lanes. The partner index moves between lanes by DPP (G <= 4),
// readlane (G = 64) or ds_bpermute. The source row x_i stays in VGPRs (or
// in LDS for very wide rows) while consecutive slots share it.
//
// Distances are computed in binary32 and compared against a band
// [lo, hi] around eps^2 that bounds the rounding error of both the binary32
// sum and the binary64 definition; a slot that falls inside the band is
// re-decided with the defining binary64 sum, so every decision equals the
// binary64 one.
#include "sng_pass_a.hpp"

namespace sng {

// Plain decision: accept iff the binary32 distance is surely below the band,
// or the binary64 recheck accepts. Accepted slots add to both degrees and set
// their accept bit (kept per call: four bits per lane, eight lanes per word).
// kQ: the query (kSimNone: the distance against eps; kSimCos: the same band
// test on the unit-scaled copy, rechecked with the binary64 cosine of the
// caller's rows; kSimDot: the dot-product filter of SimQuery).
template <int kQ>
struct PlainPolicy {
    static constexpr bool kDot = kQ == kSimDot;
    uint32_t *deg;
    uint32_t *mask;
    float lo, hi;
    double eps2;
    SimQuery sim;
    int out_deg = 0;     // 1: out-degrees (no partner-side count)
    uint32_t deg_i = 0;  // accepted slots of the cached source row
    uint32_t nib = 0;    // accept bits of this lane's own call

    __device__ __forceinline__ void begin_chunk() { nib = 0; }
    __device__ __forceinline__ void flush_source(uint32_t src, int q)
    {
        if (deg_i != 0 && q == 0)
            atomicAdd(deg + src, deg_i);
        deg_i = 0;
    }
    __device__ __forceinline__ int recheck(uint32_t i, uint32_t j, const float *rowi,
                                           const float *rowj, int d, Tally &t, int q)
    {
        t.rechecked += (q == 0);
        if constexpr (kQ == kSimNone)
            return sqdist_f64(rowi, rowj, d) <= eps2;
        else
            return sim_accept_f64(sim.X0 + (int64_t)i * sim.ld0, sim.X0 + (int64_t)j * sim.ld0, d,
                                  kQ, sim.tau);
    }
    __device__ __forceinline__ int decide(float F, uint32_t i, uint32_t j, const float *rowi,
                                          const float *rowj, int d, Tally &t, int q)
    {
        if (F <= lo)
            return 1;
        if (F > hi)
            return 0;
        return recheck(i, j, rowi, rowj, d, t, q);
    }
    __device__ __forceinline__ int decide_dot(float P, float Q, uint32_t i, uint32_t j,
                                              const float *rowi, const float *rowj, int d,
                                              Tally &t, int q)
    {
        const int r = sim.band_dot(P, Q);
        return r >= 0 ? r : recheck(i, j, rowi, rowj, d, t, q);
    }
    __device__ __forceinline__ void record(int acc, uint32_t, uint32_t j, int q, int o, int w,
                                           Tally &t)
    {
        if (acc) {
            deg_i += 1;
            if (q == 0) {
                if (!out_deg)
                    atomicAdd(deg + j, 1u);
                t.accepted += 1;
            }
            if (q == o)
                nib |= 1u << w;
        }
    }
    __device__ __forceinline__ void end_chunk(uint64_t gchunk, int lane)
    {
        if (mask) {
            const uint32_t word = or8(nib << (4 * (lane & 7)));
            if ((lane & 7) == 0)
                mask[gchunk * 8ull + (uint64_t)(lane >> 3)] = word;
        }
    }
};

template <int kQ>
__device__ __forceinline__ PlainPolicy<kQ> plain_policy(const Inst &I)
{
    PlainPolicy<kQ> p;
    p.deg = I.deg;
    p.mask = I.mask;
    p.lo = I.lo;
    p.hi = I.hi;
    p.eps2 = I.eps2;
    p.sim = I.sim;
    p.out_deg = I.out_deg;
    return p;
}

template <class Row, int OB, int kQ>
__global__ __launch_bounds__(256) void k_pass_a(Inst I, uint32_t cpw, uint32_t slice_floats)
{
    extern __shared__ float lds[];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t lo = wave * cpw;
    float *slice = lds + (threadIdx.x / kWave) * slice_floats;
    Tally t;
    PlainPolicy<kQ> pol = plain_policy<kQ>(I);
    if (lo < I.chunks)  // wave-uniform
        pass_a_range<Row, OB>(I, pol, lo, min(lo + cpw, I.chunks), slice, t);
    commit_tally(t, I.cnt);
}

// Batch form: global chunks are split at instance boundaries (each instance
// starts on a chunk of its own), so a wave looks its instance up per chunk.
template <class Row, int OB>
__global__ __launch_bounds__(256) void k_pass_a_batch(const Inst *__restrict__ table, int count,
                                                      const uint64_t *__restrict__ starts,
                                                      uint64_t total, uint32_t cpw,
                                                      uint32_t slice_floats)
{
    extern __shared__ float lds[];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    uint64_t lo = wave * cpw;
    if (lo >= total)
        return;
    const uint64_t hi = min(lo + cpw, total);
    float *slice = lds + (threadIdx.x / kWave) * slice_floats;
    while (lo < hi) {
        // instance k with starts[k] <= lo < starts[k+1]
        int a = 0, b = count - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (starts[mid] <= lo)
                a = mid;
            else
                b = mid - 1;
        }
        const Inst I = table[a];
        const uint64_t end = min(hi, starts[a + 1]);
        Tally t;
        PlainPolicy<kSimNone> pol = plain_policy<kSimNone>(I);
        pass_a_range<Row, OB>(I, pol, lo - starts[a], end - starts[a], slice, t);
        commit_tally_wave(t, I.cnt);
        lo = end;
    }
}

// ---------------------------------------------------------------------------
// Host side: pick a row policy and launch.
// ---------------------------------------------------------------------------

void band_fp32(double eps2, int d, float *lo, float *hi, double *rel)
{
    // |F - S| <= a*S + beta for the binary32 sum F of the d squared binary32
    // differences (any summation order, fused or not; beta covers flushed
    // subnormals), and |D - S| <= c*S + beta64 for the binary64 definition D,
    // S being the exact squared distance. F <= lo then forces D <= eps2 and
    // F > hi forces D > eps2.
    const double u32 = 0x1p-24, u64 = 0x1p-53;
    const double ka = (double)d + 2.0, kc = (double)d + 3.0;
    if (ka * u32 >= 0.5) {
        *lo = -1.0f;
        *hi = __builtin_inff();
        if (rel)
            *rel = __builtin_inf();
        return;
    }
    const double a = ka * u32 / (1.0 - ka * u32);
    const double c = kc * u64 / (1.0 - kc * u64);
    const double beta = (2.0 * d + 2.0) * 0x1p-126;
    const double beta64 = (2.0 * d + 2.0) * 0x1p-1074;
    double lo_r = (eps2 - beta64) * (1.0 - a) / (1.0 + c) - beta;
    double hi_r = (eps2 + beta64) * (1.0 + a) / (1.0 - c) + beta;
    lo_r -= __builtin_fabs(lo_r) * 0x1p-48;  // slack for the rounding of this arithmetic
    hi_r += __builtin_fabs(hi_r) * 0x1p-48;
    float l = (float)lo_r;
    if ((double)l > lo_r)
        l = __builtin_nextafterf(l, -__builtin_inff());
    float h = (float)hi_r;
    if ((double)h < hi_r)
        h = __builtin_nextafterf(h, __builtin_inff());
    if (lo_r < 0.0)
        l = -1.0f;
    *lo = l;
    *hi = h;
    if (rel)
        *rel = a + c;
}

PassAShape resolve_shape(int d, bool vec_ok, int lanes_req, int cpw_req, int lds_req,
                         int prefetch_req)
{
    PassAShape s;
    s.waves_per_block = 4;
    s.stage_lds = lds_req ? 1 : 0;
    int g = lanes_req;
    if (s.stage_lds) {
        g = 64;
    } else if (g <= 0) {
        if (d <= 8) {
            g = 1;
        } else {
            const int units = vec_ok ? (d + 3) / 4 : d;
            g = 1;
            while (g < units && g < 64)
                g <<= 1;
        }
    }
    if (!s.stage_lds && !vec_ok && !(g == 1 && d <= 8)) {
        // scalar row policies exist for 4, 16 and 64 lanes
        g = g <= 4 ? 4 : (g <= 16 ? 16 : 64);
    }
    s.lanes = g;
    s.chunks_per_wave = cpw_req > 0 ? cpw_req : 8;
    int ob = prefetch_req > 0 ? prefetch_req / 4 : (g >= 2 ? 2 : 1);
    ob = ob >= 4 ? 4 : (ob >= 2 ? 2 : 1);
    while (ob > g)
        ob >>= 1;
    s.owners_per_batch = ob;
    return s;
}

namespace {

template <class Row, int OB>
hipError_t go(const Inst &I, const PassAShape &sh, uint32_t slice, hipStream_t st)
{
    const uint64_t waves = (I.chunks + sh.chunks_per_wave - 1) / sh.chunks_per_wave;
    const uint64_t blocks = (waves + sh.waves_per_block - 1) / sh.waves_per_block;
    if (blocks == 0)
        return hipSuccess;
    if (blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    const size_t lds = (size_t)slice * sizeof(float) * sh.waves_per_block;
    const dim3 grid((unsigned)blocks), block(64 * sh.waves_per_block);
    const uint32_t cpw = (uint32_t)sh.chunks_per_wave;
    if (I.sim.kind == kSimDot)
        hipLaunchKernelGGL((k_pass_a<Row, OB, kSimDot>), grid, block, lds, st, I, cpw, slice);
    else if (I.sim.kind == kSimCos)
        hipLaunchKernelGGL((k_pass_a<Row, OB, kSimCos>), grid, block, lds, st, I, cpw, slice);
    else
        hipLaunchKernelGGL((k_pass_a<Row, OB, kSimNone>), grid, block, lds, st, I, cpw, slice);
    return hipGetLastError();
}

template <class Row, int OB>
hipError_t go_batch(const Inst *table, int count, const uint64_t *starts, uint64_t total,
                    const PassAShape &sh, uint32_t slice, hipStream_t st)
{
    const uint64_t waves = (total + sh.chunks_per_wave - 1) / sh.chunks_per_wave;
    const uint64_t blocks = (waves + sh.waves_per_block - 1) / sh.waves_per_block;
    if (blocks == 0)
        return hipSuccess;
    if (blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    const size_t lds = (size_t)slice * sizeof(float) * sh.waves_per_block;
    hipLaunchKernelGGL((k_pass_a_batch<Row, OB>), dim3((unsigned)blocks),
                       dim3(64 * sh.waves_per_block), lds, st, table, count, starts, total,
                       (uint32_t)sh.chunks_per_wave, slice);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pass_a(const Inst &I, const PassAShape &sh, hipStream_t st)
{
    if (I.chunks == 0)
        return hipSuccess;
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    if ((size_t)((I.d + 63) & ~63) * 4 * sh.waves_per_block > 65536 &&
        (sh.stage_lds || (!vec_ok && I.d > 16 * 64) || (vec_ok && I.d > 4 * 8 * 64)))
        return hipErrorInvalidValue;
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t slice) {
        return go<Row, OB>(I, sh, slice, st);
    });
}

hipError_t launch_pass_a_batch(const Inst *table, int count, const uint64_t *starts,
                               uint64_t total, int d, bool vec_ok, const PassAShape &sh,
                               hipStream_t st)
{
    if (total == 0)
        return hipSuccess;
    return dispatch(d, vec_ok, sh, [&]<class Row, int OB>(uint32_t slice) {
        return go_batch<Row, OB>(table, count, starts, total, sh, slice, st);
    });
}

}  // namespace sng
