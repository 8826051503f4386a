// Shared machinery of the sampled-distance passes (plain, sweep, batch).
#pragma once

#include "sng_internal.hpp"

namespace sng {

// ---------------------------------------------------------------------------
// Row policies: how a group holds x_i, fetches its share of a gathered row x_j
// into registers (fetch), and forms its partial sum of squared differences
// (partial). Fetch and partial are split so that a batch of partner rows can
// be in flight before the first distance is formed.
// ---------------------------------------------------------------------------

// G = 1, compile-time dimension D <= 8, scalar loads (any row stride).
// Dot-product query: acc.x += a*b and acc.y += |a*b| (the second bounds the
// rounding error of the first). Coordinates a row does not have are zero in
// both sums.
__device__ __forceinline__ void dot_step(float2 &acc, float a, float b)
{
    acc.x = __builtin_fmaf(a, b, acc.x);
    acc.y = __builtin_fmaf(__builtin_fabsf(a), __builtin_fabsf(b), acc.y);
}

template <int D>
struct SmallRow {
    static constexpr int kG = 1;
    static constexpr bool kPrefetch = true;
    struct Buf {
        float v[D];
    };
    Buf r;
    // A row staged in LDS as D packed floats (an LDS address, so the
    // address arithmetic stays 32-bit).
    __device__ __forceinline__ static Buf fetch_lds(const __attribute__((address_space(3))) float *row)
    {
        Buf b;
#pragma unroll
        for (int k = 0; k < D; ++k)
            b.v[k] = row[k];
        return b;
    }
    __device__ __forceinline__ static Buf fetch(const float *__restrict__ row, int, int)
    {
        Buf b;
#pragma unroll
        for (int k = 0; k < D; ++k)
            b.v[k] = row[k];
        return b;
    }
    // The same from a buffer: row at byte offset `off`.
    __device__ __forceinline__ static Buf fetchb(__amdgpu_buffer_rsrc_t rs, uint32_t off, int, int)
    {
        Buf b;
        if constexpr (D == 3) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, (int)off, 0, 0);
            b.v[0] = __uint_as_float(v[0]);
            b.v[1] = __uint_as_float(v[1]);
            b.v[2] = __uint_as_float(v[2]);
        } else if constexpr (D == 2) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
            b.v[0] = __uint_as_float(v[0]);
            b.v[1] = __uint_as_float(v[1]);
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k)
                b.v[k] = bld1(rs, off + 4u * k);
        }
        return b;
    }
    __device__ __forceinline__ void load(const float *row, int q, int d, float *)
    {
        r = fetch(row, q, d);
    }
    __device__ __forceinline__ float partial(const Buf &b, int, int) const
    {
        return partial2(r, b, 0, D);
    }
    __device__ __forceinline__ static float partial2(const Buf &a, const Buf &b, int, int)
    {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float e = a.v[k] - b.v[k];
            acc = __builtin_fmaf(e, e, acc);
        }
        return acc;
    }
    __device__ __forceinline__ float2 partial_dot(const Buf &b, int, int) const
    {
        return partial2_dot(r, b, 0, D);
    }
    __device__ __forceinline__ static float2 partial2_dot(const Buf &a, const Buf &b, int, int)
    {
        float2 acc = {0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < D; ++k)
            dot_step(acc, a.v[k], b.v[k]);
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
    __device__ __forceinline__ static Buf fetchb(__amdgpu_buffer_rsrc_t rs, uint32_t off, int q,
                                                 int d)
    {
        Buf b;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int k = 4 * (v * G + q);
            if (FULL || k < d)
                b.v[v] = bld4(rs, off + 4u * (uint32_t)k);
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
        return partial2(r, b, q, d);
    }
    __device__ __forceinline__ static float partial2(const Buf &a, const Buf &b, int q, int d)
    {
        float acc = 0.0f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int k = 4 * (v * G + q);
            const float e0 = a.v[v].x - b.v[v].x;
            const float e1 = (FULL || k + 1 < d) ? a.v[v].y - b.v[v].y : 0.0f;
            const float e2 = (FULL || k + 2 < d) ? a.v[v].z - b.v[v].z : 0.0f;
            const float e3 = (FULL || k + 3 < d) ? a.v[v].w - b.v[v].w : 0.0f;
            acc = __builtin_fmaf(e0, e0, acc);
            acc = __builtin_fmaf(e1, e1, acc);
            acc = __builtin_fmaf(e2, e2, acc);
            acc = __builtin_fmaf(e3, e3, acc);
        }
        return acc;
    }
    __device__ __forceinline__ float2 partial_dot(const Buf &b, int q, int d) const
    {
        return partial2_dot(r, b, q, d);
    }
    __device__ __forceinline__ static float2 partial2_dot(const Buf &a, const Buf &b, int q, int d)
    {
        float2 acc = {0.0f, 0.0f};
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int k = 4 * (v * G + q);
            dot_step(acc, a.v[v].x, b.v[v].x);
            if (FULL || k + 1 < d)
                dot_step(acc, a.v[v].y, b.v[v].y);
            if (FULL || k + 2 < d)
                dot_step(acc, a.v[v].z, b.v[v].z);
            if (FULL || k + 3 < d)
                dot_step(acc, a.v[v].w, b.v[v].w);
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
    __device__ __forceinline__ static Buf fetchb(__amdgpu_buffer_rsrc_t rs, uint32_t off, int q,
                                                 int d)
    {
        Buf b;
#pragma unroll
        for (int v = 0; v < NS; ++v) {
            const int k = v * G + q;
            b.v[v] = (k < d) ? bld1(rs, off + 4u * (uint32_t)k) : 0.0f;
        }
        return b;
    }
    __device__ __forceinline__ void load(const float *row, int q, int d, float *)
    {
        r = fetch(row, q, d);
    }
    __device__ __forceinline__ float partial(const Buf &b, int q, int d) const
    {
        return partial2(r, b, q, d);
    }
    __device__ __forceinline__ static float partial2(const Buf &a, const Buf &b, int, int)
    {
        float acc = 0.0f;
#pragma unroll
        for (int v = 0; v < NS; ++v) {
            const float e = a.v[v] - b.v[v];
            acc = __builtin_fmaf(e, e, acc);
        }
        return acc;
    }
    __device__ __forceinline__ float2 partial_dot(const Buf &b, int q, int d) const
    {
        return partial2_dot(r, b, q, d);
    }
    __device__ __forceinline__ static float2 partial2_dot(const Buf &a, const Buf &b, int, int)
    {
        float2 acc = {0.0f, 0.0f};
#pragma unroll
        for (int v = 0; v < NS; ++v)
            dot_step(acc, a.v[v], b.v[v]);
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
    __device__ __forceinline__ float2 partial_dot(const Buf &b, int q, int d) const
    {
        float2 acc = {0.0f, 0.0f};
        for (int k = q; k < d; k += 64)
            dot_step(acc, s[k], b.p[k]);
        return acc;
    }
};

// Per-lane tallies, summed into the workspace counters at the end.
struct Tally {
    uint32_t self = 0, accepted = 0, rechecked = 0;
};

// Walks local chunks [ch_lo, ch_hi) of instance I: every lane computes one
// Philox call (four slots), every group of G lanes evaluates the 4G slots of
// its own G calls. OB calls of a group are handled per batch: their 4*OB
// partner rows are fetched first, then decided one after another. What a
// decision is, and what it updates, is the policy's business (Pol):
//   begin_chunk()                 per chunk, before any slot
//   flush_source(src, q)          the group leaves source row src
//   decide(F, i, j, rowi, rowj, d, t, q)  group-uniform result for one slot
//                                 from its binary32 squared distance F, or
//   decide_dot(P, Q, i, j, ...)   from its binary32 dot product P and sum of
//                                 absolute products Q when Pol::kDot
//   record(r, i, j, q, o, w, t)   account one decided slot (call o, word w)
//   end_chunk(global_chunk, lane) per chunk, after every slot
// Every cross-lane operation happens under group-uniform control flow.
template <class Row, int OB, class Pol>
__device__ __forceinline__ void pass_a_range(const Inst &I, Pol &pol, uint64_t ch_lo,
                                             uint64_t ch_hi, float *slice, Tally &tally)
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

    Row xi;
    uint32_t cached = 0xFFFFFFFFu;  // source row held by the group
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
        partners4(I, W, j);

        pol.begin_chunk();
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
                if (io[b] != cached) {
                    if (cached != 0xFFFFFFFFu)
                        pol.flush_source(cached, q);
                    xi.load(X + (int64_t)io[b] * ld, q, d, slice);
                    cached = io[b];
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
                    int r;
                    if constexpr (Pol::kDot) {
                        const float2 pq = xi.partial_dot(buf[b][w], q, d);
                        const float P = group_all<G>(group_sum<G>(pq.x));
                        const float Q = group_all<G>(group_sum<G>(pq.y));
                        r = pol.decide_dot(P, Q, io[b], jw, X + (int64_t)io[b] * ld, rowj, d,
                                           tally, q);
                    } else {
                        const float F = group_all<G>(group_sum<G>(xi.partial(buf[b][w], q, d)));
                        r = pol.decide(F, io[b], jw, X + (int64_t)io[b] * ld, rowj, d, tally, q);
                    }
                    pol.record(r, io[b], jw, q, o, w, tally);
                }
            }
        }
        pol.end_chunk(I.chunk0 + ch, lane);
        c0 += 64u;
        if (c0 >= I.C) {
            const uint32_t k = div_exact(c0, I.C, I.inv_C);
            i0 += k;
            c0 -= k * I.C;
        }
    }
    if (cached != 0xFFFFFFFFu)
        pol.flush_source(cached, q);
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

// Calls fn.template operator()<Row, OB>(slice) for the policy of (d, shape).
template <class Row, class Fn>
inline hipError_t with_ob(const PassAShape &sh, uint32_t slice, Fn &&fn)
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
inline hipError_t dispatch(int d, bool vec_ok, const PassAShape &sh, Fn &&fn)
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

}  // namespace sng
