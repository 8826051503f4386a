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
#include "sng_internal.hpp"

namespace sng {

// ---------------------------------------------------------------------------
// Row policies: how a group holds x_i, fetches its share of a gathered row x_j
// into registers (fetch), and forms its partial sum of squared differences
// (partial). Fetch and partial are split so that a batch of partner rows can
// be in flight before the first distance is formed.
// ---------------------------------------------------------------------------

// G = 1, compile-time dimension D <= 8, scalar loads (any row stride).
template <int D>
struct SmallRow {
    static constexpr int kG = 1;
    static constexpr bool kPrefetch = true;
    struct Buf {
        float v[D];
    };
    Buf r;
    __device__ __forceinline__ static Buf fetch(const float *__restrict__ row, int, int)
    {
        Buf b;
#pragma unroll
        for (int k = 0; k < D; ++k)
            b.v[k] = row[k];
        return b;
    }
    __device__ __forceinline__ void load(const float *row, int q, int d, float *)
    {
        r = fetch(row, q, d);
    }
    __device__ __forceinline__ float partial(const Buf &b, int, int) const
    {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float e = r.v[k] - b.v[k];
            acc = __builtin_fmaf(e, e, acc);
        }
        return acc;
    }
};

// G lanes, NV float4 per lane: lane q holds coordinates 4*(v*G + q) + 0..3.
// Requires 16-byte aligned rows. FULL: d == 4*G*NV (no tail masking).
template <int G, int NV, bool FULL>
struct VecRow {
    static constexpr int kG = G;
    static constexpr bool kPrefetch = true;
    struct Buf {
        float4 v[NV];
    };
    Buf r;
    __device__ __forceinline__ static Buf fetch(const float *__restrict__ row, int q, int d)
    {
        Buf b;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int k = 4 * (v * G + q);
            if (FULL || k < d)
                b.v[v] = *reinterpret_cast<const float4 *>(row + k);
            else
                b.v[v] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return b;
    }
    __device__ __forceinline__ void load(const float *row, int q, int d, float *)
    {
        r = fetch(row, q, d);
    }
    __device__ __forceinline__ float partial(const Buf &b, int q, int d) const
    {
        float acc = 0.0f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int k = 4 * (v * G + q);
            const float e0 = r.v[v].x - b.v[v].x;
            const float e1 = (FULL || k + 1 < d) ? r.v[v].y - b.v[v].y : 0.0f;
            const float e2 = (FULL || k + 2 < d) ? r.v[v].z - b.v[v].z : 0.0f;
            const float e3 = (FULL || k + 3 < d) ? r.v[v].w - b.v[v].w : 0.0f;
            acc = __builtin_fmaf(e0, e0, acc);
            acc = __builtin_fmaf(e1, e1, acc);
            acc = __builtin_fmaf(e2, e2, acc);
            acc = __builtin_fmaf(e3, e3, acc);
        }
        return acc;
    }
};

// G lanes, NS scalars per lane: lane q holds coordinates v*G + q. Any row
// stride and alignment.
template <int G, int NS>
struct ScalarRow {
    static constexpr int kG = G;
    static constexpr bool kPrefetch = true;
    struct Buf {
        float v[NS];
    };
    Buf r;
    __device__ __forceinline__ static Buf fetch(const float *__restrict__ row, int q, int d)
    {
        Buf b;
#pragma unroll
        for (int v = 0; v < NS; ++v) {
            const int k = v * G + q;
            b.v[v] = (k < d) ? row[k] : 0.0f;
        }
        return b;
    }
    __device__ __forceinline__ void load(const float *row, int q, int d, float *)
    {
        r = fetch(row, q, d);
    }
    __device__ __forceinline__ float partial(const Buf &b, int, int) const
    {
        float acc = 0.0f;
#pragma unroll
        for (int v = 0; v < NS; ++v) {
            const float e = r.v[v] - b.v[v];
            acc = __builtin_fmaf(e, e, acc);
        }
        return acc;
    }
};

// G = 64: the source row is staged in this wave's LDS slice (any d that fits);
// the partner row is streamed from memory while the distance is formed.
struct LdsRow {
    static constexpr int kG = 64;
    static constexpr bool kPrefetch = false;
    struct Buf {
        const float *p;
    };
    float *s = nullptr;
    __device__ __forceinline__ static Buf fetch(const float *row, int, int) { return Buf{row}; }
    __device__ __forceinline__ void load(const float *row, int q, int d, float *slice)
    {
        s = slice;
        __builtin_amdgcn_wave_barrier();
        for (int k = q; k < d; k += 64)
            s[k] = row[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ __forceinline__ float partial(const Buf &b, int q, int d) const
    {
        float acc = 0.0f;
        for (int k = q; k < d; k += 64) {
            const float e = s[k] - b.p[k];
            acc = __builtin_fmaf(e, e, acc);
        }
        return acc;
    }
};

// Per-lane tallies, summed into the workspace counters at the end.
struct Tally {
    uint32_t self = 0, accepted = 0, rechecked = 0;
};

// The group's running state across candidates: which source row is cached
// and how many of its slots were accepted since the last flush.
template <class Row>
struct GroupState {
    Row xi;
    uint32_t cached = 0xFFFFFFFFu;
    uint32_t deg_i = 0;
};

template <class Row>
__device__ __forceinline__ void flush_source(GroupState<Row> &gs, uint32_t *deg, int q)
{
    if (gs.deg_i != 0 && q == 0)
        atomicAdd(deg + gs.cached, gs.deg_i);
    gs.deg_i = 0;
}

// Processes local chunks [ch_lo, ch_hi) of instance I. OB owners (calls) of
// a group are handled per batch: their 4*OB partner rows are fetched first,
// then decided one after another.
template <class Row, int OB>
__device__ __forceinline__ void pass_a_range(const Inst &I, uint64_t ch_lo, uint64_t ch_hi,
                                             float *slice, Tally &tally)
{
    constexpr int G = Row::kG;
    static_assert(OB >= 1 && OB <= G, "owners per batch");
    const int lane = lane_id();
    const int q = lane & (G - 1);
    const float *__restrict__ X = I.X;
    const int64_t ld = I.ld;
    const int d = I.d;

    // (source, call) of lane 0's call in the first chunk
    const uint64_t call0 = ch_lo * 64ull;
    uint32_t i0 = (uint32_t)(call0 / I.C);
    uint32_t c0 = (uint32_t)(call0 - (uint64_t)i0 * I.C);

    GroupState<Row> gs;
    for (uint64_t ch = ch_lo; ch < ch_hi; ++ch) {
        uint32_t cc = c0 + (uint32_t)lane;
        uint32_t ii = i0;
        if (cc >= I.C) {
            const uint32_t k = div_exact(cc, I.C, I.inv_C);
            ii += k;
            cc -= k * I.C;
        }
        const uint32_t nvalid = (ii < I.n) ? min(4u, I.m - 4u * cc) : 0u;
        const Words4 W = philox10(cc, ii, I.key0, I.key1);
        uint32_t j[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            j[w] = mod_exact(W.w[w], I.n, I.inv_n);

        uint32_t nib = 0;  // accept bits of this lane's own call
        constexpr int kBatches = G / OB;
        constexpr int kBatchUnroll = (G <= 4) ? kBatches : 1;
#pragma unroll kBatchUnroll
        for (int ob = 0; ob < kBatches; ++ob) {
            uint32_t io[OB], nv[OB], jj[OB][4];
            typename Row::Buf buf[OB][4];
#pragma unroll
            for (int b = 0; b < OB; ++b) {
                const int o = ob * OB + b;
                io[b] = group_bcast<G>(ii, o);
                nv[b] = group_bcast<G>(nvalid, o);
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    jj[b][w] = group_bcast<G>(j[w], o);
            }
            if constexpr (Row::kPrefetch) {
                // Issue every partner gather of the batch before using any.
#pragma unroll
                for (int b = 0; b < OB; ++b)
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const bool live = (uint32_t)w < nv[b] && jj[b][w] != io[b];
                        const uint32_t src = live ? jj[b][w] : 0u;  // row 0 always exists
                        buf[b][w] = Row::fetch(X + (int64_t)src * ld, q, d);
                    }
            }
#pragma unroll
            for (int b = 0; b < OB; ++b) {
                const int o = ob * OB + b;
                if (nv[b] == 0)
                    continue;  // call beyond n (group-uniform)
                if (io[b] != gs.cached) {
                    flush_source(gs, I.deg, q);
                    gs.xi.load(X + (int64_t)io[b] * ld, q, d, slice);
                    gs.cached = io[b];
                }
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if ((uint32_t)w >= nv[b])
                        continue;  // slot beyond m (group-uniform)
                    const uint32_t jw = jj[b][w];
                    if (jw == io[b]) {
                        tally.self += (q == 0);
                        continue;
                    }
                    const float *rowj = X + (int64_t)jw * ld;
                    if constexpr (!Row::kPrefetch)
                        buf[b][w] = Row::fetch(rowj, q, d);
                    float F = group_sum<G>(gs.xi.partial(buf[b][w], q, d));
                    F = __int_as_float((int)group_bcast<G>((uint32_t)__float_as_int(F), 0));
                    bool acc;
                    if (F <= I.lo) {
                        acc = true;
                    } else if (F > I.hi) {
                        acc = false;
                    } else {
                        const double D = sqdist_f64(X + (int64_t)io[b] * ld, rowj, d);
                        acc = (D <= I.eps2);
                        tally.rechecked += (q == 0);
                    }
                    if (acc) {
                        gs.deg_i += 1;
                        if (q == 0) {
                            atomicAdd(I.deg + jw, 1u);
                            tally.accepted += 1;
                        }
                        if (q == o)
                            nib |= 1u << w;
                    }
                }
            }
        }
        if (I.mask) {
            const uint32_t word = or8(nib << (4 * (lane & 7)));
            if ((lane & 7) == 0)
                I.mask[(I.chunk0 + ch) * 8ull + (uint64_t)(lane >> 3)] = word;
        }
        c0 += 64u;
        if (c0 >= I.C) {
            const uint32_t k = div_exact(c0, I.C, I.inv_C);
            i0 += k;
            c0 -= k * I.C;
        }
    }
    if (gs.cached != 0xFFFFFFFFu)
        flush_source(gs, I.deg, q);
}

// One atomic per wave and counter (used where waves of a block work for
// different instances).
__device__ __forceinline__ void commit_tally_wave(const Tally &t, unsigned long long *cnt)
{
    if (!cnt)
        return;
    const unsigned long long s = wave_sum_u64(t.self);
    const unsigned long long a = wave_sum_u64(t.accepted);
    const unsigned long long r = wave_sum_u64(t.rechecked);
    if (lane_id() == 0) {
        if (s) atomicAdd(cnt + kCntSelf, s);
        if (a) atomicAdd(cnt + kCntAccepted, a);
        if (r) atomicAdd(cnt + kCntRechecked, r);
    }
}

// One atomic per block and counter (all threads of the block call this).
__device__ __forceinline__ void commit_tally(const Tally &t, unsigned long long *cnt)
{
    const int slots[3] = {kCntSelf, kCntAccepted, kCntRechecked};
    const uint32_t v[3] = {t.self, t.accepted, t.rechecked};
    block_count_add<3>(cnt, slots, v);
}

template <class Row, int OB>
__global__ __launch_bounds__(256) void k_pass_a(Inst I, uint32_t cpw, uint32_t slice_floats)
{
    extern __shared__ float lds[];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t lo = wave * cpw;
    float *slice = lds + (threadIdx.x / kWave) * slice_floats;
    Tally t;
    if (lo < I.chunks)  // wave-uniform
        pass_a_range<Row, OB>(I, lo, min(lo + cpw, I.chunks), slice, t);
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
        pass_a_range<Row, OB>(I, lo - starts[a], end - starts[a], slice, t);
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
    hipLaunchKernelGGL((k_pass_a<Row, OB>), dim3((unsigned)blocks), dim3(64 * sh.waves_per_block),
                       lds, st, I, (uint32_t)sh.chunks_per_wave, slice);
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

// Calls fn.template operator()<Row, OB>(slice) for the policy of (d, shape).
template <class Row, class Fn>
hipError_t with_ob(const PassAShape &sh, uint32_t slice, Fn &&fn)
{
    constexpr int G = Row::kG;
    if constexpr (G >= 4) {
        if (sh.owners_per_batch >= 4)
            return fn.template operator()<Row, 4>(slice);
    }
    if constexpr (G >= 2) {
        if (sh.owners_per_batch >= 2)
            return fn.template operator()<Row, 2>(slice);
    }
    return fn.template operator()<Row, 1>(slice);
}

template <class Fn>
hipError_t dispatch(int d, bool vec_ok, const PassAShape &sh, Fn &&fn)
{
    const int G = sh.lanes;
    const uint32_t lds_slice = (uint32_t)((d + 63) & ~63);
    if (sh.stage_lds)
        return fn.template operator()<LdsRow, 1>(lds_slice);
    if (d <= 8 && G == 1) {
        switch (d) {
        case 1: return fn.template operator()<SmallRow<1>, 1>(0u);
        case 2: return fn.template operator()<SmallRow<2>, 1>(0u);
        case 3: return fn.template operator()<SmallRow<3>, 1>(0u);
        case 4: return fn.template operator()<SmallRow<4>, 1>(0u);
        case 5: return fn.template operator()<SmallRow<5>, 1>(0u);
        case 6: return fn.template operator()<SmallRow<6>, 1>(0u);
        case 7: return fn.template operator()<SmallRow<7>, 1>(0u);
        default: return fn.template operator()<SmallRow<8>, 1>(0u);
        }
    }
    if (vec_ok) {
        const int units = (d + 3) / 4;
        const int nv = (units + G - 1) / G;
        const bool full = (d == 4 * G * nv);
#define SNG_VEC(GG)                                                                          \
    if (G == GG) {                                                                           \
        if (nv == 1)                                                                         \
            return full ? with_ob<VecRow<GG, 1, true>>(sh, 0u, fn)                           \
                        : with_ob<VecRow<GG, 1, false>>(sh, 0u, fn);                         \
        if (nv == 2) return with_ob<VecRow<GG, 2, false>>(sh, 0u, fn);                       \
        if (nv <= 4) return fn.template operator()<VecRow<GG, 4, false>, 1>(0u);             \
        if (nv <= 8) return fn.template operator()<VecRow<GG, 8, false>, 1>(0u);             \
    }
        SNG_VEC(1)
        SNG_VEC(2)
        SNG_VEC(4)
        SNG_VEC(8)
        SNG_VEC(16)
        SNG_VEC(32)
        SNG_VEC(64)
#undef SNG_VEC
    } else {
        const int ns = (d + G - 1) / G;
#define SNG_SCA(GG)                                                                          \
    if (G == GG) {                                                                           \
        if (ns <= 1) return fn.template operator()<ScalarRow<GG, 1>, 1>(0u);                 \
        if (ns <= 2) return fn.template operator()<ScalarRow<GG, 2>, 1>(0u);                 \
        if (ns <= 4) return fn.template operator()<ScalarRow<GG, 4>, 1>(0u);                 \
        if (ns <= 8) return fn.template operator()<ScalarRow<GG, 8>, 1>(0u);                 \
        if (ns <= 16) return fn.template operator()<ScalarRow<GG, 16>, 1>(0u);               \
    }
        SNG_SCA(4)
        SNG_SCA(16)
        SNG_SCA(64)
#undef SNG_SCA
    }
    // anything else: LDS-staged wave-per-pair
    return fn.template operator()<LdsRow, 1>(lds_slice);
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
