// Evaluate kernels of the partner-block schedule (see sng_bucket.hip for the
// schedule): the decision policies, the ticket walk and the kernels, shared
// by the translation units that instantiate them (one per query, so they
// compile in parallel).
#pragma once

#include "sng_pass_a.hpp"

namespace sng {

constexpr uint32_t kRecOffShift = 18;  // record: call offset (14 bits) | word (2) | partner (16)

// Decisions take point indices; row pointers for the binary64 recheck are
// formed only inside the band. record() receives the slot's global call
// number as a functor, evaluated only for accepted slots. kQ: the query, as
// for the direct pass (kSimCos evaluates the unit-scaled copy in X and
// rechecks the caller's rows; kSimDot uses the dot-product filter).
template <int kQ>
struct BucketPlainPolicy {
    static constexpr bool kDot = kQ == kSimDot;
    int out_deg;  // 1: out-degrees (no partner-side count)
    const float *X;
    int64_t ld;
    int d;
    uint32_t *deg;
    uint32_t *mask;
    float lo, hi;
    double eps2;
    SimQuery sim;

    __device__ __forceinline__ int recheck(uint32_t i, uint32_t j, Tally &t, int q)
    {
        t.rechecked += (q == 0);
        if constexpr (kQ == kSimNone)
            return sqdist_f64(X + (int64_t)i * ld, X + (int64_t)j * ld, d) <= eps2;
        else
            return sim_accept_f64(sim.X0 + (int64_t)i * sim.ld0, sim.X0 + (int64_t)j * sim.ld0, d,
                                  kQ, sim.tau);
    }
    __device__ __forceinline__ int decide(float F, uint32_t i, uint32_t j, Tally &t, int q)
    {
        if (F <= lo)
            return 1;
        if (F > hi)
            return 0;
        return recheck(i, j, t, q);
    }
    // false only where decide() surely rejects (so record() does nothing)
    __device__ __forceinline__ bool may_act(float F) const { return !(F > hi); }
    __device__ __forceinline__ bool may_act_dot(float P, float Q) const
    {
        return sim.band_dot(P, Q) != 0;
    }
    __device__ __forceinline__ int decide_dot(float P, float Q, uint32_t i, uint32_t j, Tally &t,
                                              int q)
    {
        const int r = sim.band_dot(P, Q);
        return r >= 0 ? r : recheck(i, j, t, q);
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
    static constexpr bool kDot = false;

    // false only where decide() surely returns K (so record() does nothing)
    __device__ __forceinline__ bool may_act(float F) const { return F <= hi_max; }
    __device__ __forceinline__ bool may_act_dot(float, float) const { return true; }

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
            int res;
            if constexpr (Pol::kDot) {
                const float2 pq = Row::partial2_dot(bi[k], bj[k], q, d);
                const float P = group_all<G>(group_sum<G>(pq.x));
                const float Q = group_all<G>(group_sum<G>(pq.y));
                res = pol.decide_dot(P, Q, ii[k], cj[k], tally, q);
            } else {
                const float F = group_all<G>(group_sum<G>(Row::partial2(bi[k], bj[k], q, d)));
                res = pol.decide(F, ii[k], cj[k], tally, q);
            }
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

template <class Row, int OB, bool kBuf, int kQ>
__global__ __launch_bounds__(256) void k_bkt_eval_plain(Inst I, BucketGeom B)
{
    if (!sample_ok(I, B))
        return;
    BucketPlainPolicy<kQ> pol;
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
// LDS form, for rows of at most kLdsMaxD floats (blocks of at most
// kLdsBlockBytes). One workgroup per compute unit takes work items (chunk of
// kLdsChunkRanges generator ranges, partner block J) from a global counter in
// chunk-major order, stages block J whole in LDS with coalesced loads, and
// its wavefronts decide every record of the item's ranges for that block:
// wavefront w takes tickets of kLdsTicketRanges ranges w, w + waves, ... .
// Partner rows are then LDS reads instead of divergent global gathers; the
// source rows of a ticket are few and consecutive (a range covers
// kRangeCalls / ceil(m/4) points), so their global loads stay coalesced, and
// the chunk-major order keeps a chunk's source rows in L2 while its blocks
// are visited.
// ---------------------------------------------------------------------------
constexpr uint32_t kLdsThreads = 1024;
constexpr uint32_t kLdsWaves = kLdsThreads / kWave;
constexpr uint32_t kLdsTicketRanges = 64;
constexpr uint64_t kLdsChunkRanges = 32768;
constexpr int kLdsWindows = 4;  // windows decided per iteration of a wavefront
static_assert(kLdsTicketRanges <= kWave, "one lane per segment of a ticket");

// One ticket of the LDS form: the records of partner block J from T <= 64
// consecutive ranges (segments), one lane per pair. Each segment is cut into
// windows of up to 64 records (a segment holds about kRangeCalls*4/NJ
// records, so most take one window), and a window's record base, first
// source and record count are scalars. A table of up to 64 windows sits one
// window per lane (each lane finds its segment by a binary search over the
// segments' window prefix); the wavefront decides P windows per iteration,
// reading their entries with readlane, and loads the next P windows' records
// (and source rows) before deciding the current ones. The partner row is
// read from `blk`, the staged block. Records carry the source's offset within
// its range and the call within the point as bit fields (BucketGeom::lds),
// so a source index is one add. kLaneRows (the rows of every range's
// sources hold at most 64 elements): lane t holds element t mod D of source
// row i0 + t / D of a window's segment, loaded with one coalesced dword load,
// and each lane takes its source row from there by D cross-lane permutes;
// otherwise each lane loads its source row. Every
// record is filtered in binary32 first, and the decision and bookkeeping run
// only when some lane may accept or must recheck, so windows of rejections
// cost the filter alone.
template <int D, int P, bool kBuf, bool kLaneRows, class Pol>
__device__ __forceinline__ void eval_ticket_lds(const Inst &I, const BucketGeom &B, Pol &pol,
                                                uint64_t r0, uint32_t T, uint32_t J,
                                                Tally &tally, const float *blk)
{
    using Row = SmallRow<D>;
    using Buf = typename Row::Buf;
    const int lane = lane_id();
    const __amdgpu_buffer_rsrc_t rrec =
        buf_rsrc(B.rec + r0 * B.region, (uint32_t)(T * B.region * sizeof(uint32_t)));
    uint32_t cnt_l = 0, i0_l = 0, base_l = 0;
    if ((uint32_t)lane < T) {
        const uint64_t r = r0 + (uint64_t)lane;
        base_l = (uint32_t)lane * (uint32_t)B.region + B.seg[(r * B.NJ + J) * 2 + 0];
        cnt_l = B.seg[(r * B.NJ + J) * 2 + 1];
        i0_l = B.start[2 * r + 0];
    }
    // windows of each segment and their inclusive prefix over the segments
    const uint32_t wc_l = (cnt_l + (uint32_t)kWave - 1) / (uint32_t)kWave;
    uint32_t winc = wc_l;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const uint32_t u = __shfl_up(winc, s);
        if (lane >= s)
            winc += u;
    }
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)winc, kWave - 1);
    if (total == 0)
        return;  // wave-uniform
    const uint32_t wexcl_l = winc - wc_l;

    const uint32_t jbase = J << B.bshift;
    const uint32_t pmask = (1u << B.bshift) - 1u;
    const uint32_t si_shift = B.bshift + 2 + B.tc_bits;
    const auto *lblk = (const __attribute__((address_space(3))) float *)blk;
    const float *__restrict__ X = I.X;
    const int64_t ld = I.ld;
    const uint32_t ld4 = (uint32_t)ld * 4u;
    __amdgpu_buffer_rsrc_t rs;
    if constexpr (kBuf)
        rs = buf_rsrc(X, B.x_bytes);
    auto row_at = [&](uint32_t r) -> Buf {
        if constexpr (kBuf)
            return Row::fetchb(rs, __umul24(r, ld4), 0, D);
        else
            return Row::fetch(X + (int64_t)r * ld, 0, D);
    };

    // the window table of windows [wb, wb + 64): lane w holds window wb + w,
    // its record base and (first source << 7 | record count); sources are
    // below n <= kMaxPartnerBlocks * 2^15 = 2^25 in this form
    uint32_t t_rec = 0, t_sn = 0;
    auto build = [&](uint32_t wb) {
        const uint32_t w = wb + (uint32_t)lane;
        // its segment: the first l with winc_l > w (winc is non-decreasing)
        uint32_t sg = 0;
#pragma unroll
        for (uint32_t step = 32; step > 0; step >>= 1) {
            const uint32_t e = (uint32_t)__builtin_amdgcn_ds_bpermute(
                (int)((sg + step - 1) << 2), (int)winc);
            sg += (e <= w) ? step : 0u;
        }
        sg &= 63u;
        const uint32_t a = sg << 2;
        const uint32_t o = (w - (uint32_t)__builtin_amdgcn_ds_bpermute((int)a, (int)wexcl_l)) *
                           (uint32_t)kWave;
        const uint32_t c = (uint32_t)__builtin_amdgcn_ds_bpermute((int)a, (int)cnt_l);
        t_rec = (uint32_t)__builtin_amdgcn_ds_bpermute((int)a, (int)base_l) + o;
        const uint32_t src = (uint32_t)__builtin_amdgcn_ds_bpermute((int)a, (int)i0_l);
        t_sn = (src << 7) | ((w < total && c > o) ? min(c - o, (uint32_t)kWave) : 0u);
    };
    // window k's entries (k in the current table)
    uint32_t wb = 0;
    build(0);
    uint32_t w_rec[P], w_src[P], w_n[P];
    auto take = [&](uint32_t k0) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int at = (int)(k0 + (uint32_t)k - wb);  // < 64 (tables are rebuilt first)
            w_rec[k] = (uint32_t)__builtin_amdgcn_readlane((int)t_rec, at);
            const uint32_t sn = (uint32_t)__builtin_amdgcn_readlane((int)t_sn, at);
            w_src[k] = sn >> 7;
            w_n[k] = sn & 127u;
        }
    };
    // kLaneRows: lane t holds element t mod D of source row src + t / D
    // (rows src .. src + 64/D - 1 cover every source of a range)
    const uint32_t lr_row = (uint32_t)lane / (uint32_t)D;
    const uint32_t lr_el = (uint32_t)lane - lr_row * (uint32_t)D;
    // The loads of P windows: records, and with kLaneRows the source rows.
    struct Win {
        uint32_t v[P], src[P], n[P];
        float row[P];
    };
    // Lanes past a window's records, and (kLaneRows) past the rows a range
    // can touch, load nothing: their buffer offset is out of range, which
    // reads zero without a memory request.
    constexpr uint32_t kNoLoad = 0xFFFFFFF0u;
    const uint32_t lr_lanes = ((I.C - 1u + (uint32_t)kRangeCalls - 1u) / I.C + 1u) * (uint32_t)D;
    auto issue = [&](Win &S) {  // windows in w_* (harmless loads for empty ones)
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if constexpr (kLaneRows) {
                const uint32_t r = w_src[k] + lr_row;
                if constexpr (kBuf) {
                    // rows past the last one read as zero through the buffer
                    S.row[k] = bld1(rs, (uint32_t)lane < lr_lanes
                                            ? __umul24(lr_row, ld4) + w_src[k] * ld4 + lr_el * 4u
                                            : kNoLoad);
                } else {
                    S.row[k] = X[(int64_t)(r < I.n ? r : I.n - 1u) * ld + lr_el];
                }
            }
            S.v[k] = __builtin_amdgcn_raw_buffer_load_b32(
                rrec, (int)((uint32_t)lane < w_n[k] ? (w_rec[k] + lane) * 4u : kNoLoad), 0, 0);
            S.src[k] = w_src[k];
            S.n[k] = w_n[k];
        }
    };
    // windows k1 .. k1 + P - 1 into w_* (a new table every 64 windows;
    // windows past the last have no records)
    auto next = [&](uint32_t k1) {
        if (k1 - wb >= (uint32_t)kWave && k1 < total) {
            wb = k1;
            build(wb);
        }
        take(k1 < total ? k1 : wb);
        if (k1 >= total) {
#pragma unroll
            for (int k = 0; k < P; ++k)
                w_n[k] = 0;
        }
    };
    static_assert(kWave % P == 0, "windows per iteration divide the table");
    // kDepth sets of windows load ahead: windows k0 + P .. k0 + kDepth*P are
    // in flight while windows k0 are decided (two sets where the registers
    // allow). A step takes the windows of its set (already loaded), reloads
    // the set with the windows kDepth steps on, then decides.
    constexpr int kDepth = D <= 5 ? 2 : 1;
    auto step = [&](Win &S, uint32_t k0) {
        uint32_t v[P], c_src[P], c_n[P];
        float crow[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            v[k] = S.v[k];
            crow[k] = S.row[k];
            c_src[k] = S.src[k];
            c_n[k] = S.n[k];
        }
        next(k0 + kDepth * P);
        issue(S);

        uint32_t ii[P], cj[P];
        Buf bi[P], bj[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint32_t so = v[k] >> si_shift;
            ii[k] = c_src[k] + so;
            const uint32_t off = v[k] & pmask;
            cj[k] = jbase + off;
            if constexpr (kLaneRows) {
                // the permutes read lanes so*D + e mod 64 (any lane: a bad so
                // is caught before a decision)
                const uint32_t a = __umul24(so, 4u * (uint32_t)D);
#pragma unroll
                for (int e = 0; e < D; ++e)
                    bi[k].v[e] = __int_as_float(
                        __builtin_amdgcn_ds_bpermute((int)(a + 4u * e), __float_as_int(crow[k])));
            } else {
                // rows past X read as zero through the buffer; the plain
                // form clamps the index (a bad one is caught before a decision)
                bi[k] = row_at(kBuf ? ii[k] : min(ii[k], I.n - 1u));
            }
            // off < 2^bshift rows: inside the block's LDS whether staged or not
            bj[k] = Row::fetch_lds(lblk + __umul24(off, (uint32_t)D));
        }
        float F[P], Q[P];
        uint64_t act = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const bool live = (uint32_t)lane < c_n[k];
            if constexpr (Pol::kDot) {
                const float2 pq = Row::partial2_dot(bi[k], bj[k], 0, D);
                F[k] = pq.x;
                Q[k] = pq.y;
                act |= __ballot(live && pol.may_act_dot(F[k], Q[k]));
            } else {
                F[k] = Row::partial2(bi[k], bj[k], 0, D);
                Q[k] = 0.0f;
                act |= __ballot(live && pol.may_act(F[k]));
            }
        }
        if (act == 0)
            return;  // wave-uniform: every live slot here is surely rejected
        // Records outside the instance (never for a valid sample) are counted
        // and their windows dropped before anything is written.
        bool live[P], bad = false;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            live[k] = (uint32_t)lane < c_n[k];
            bad |= live[k] & ((ii[k] >= I.n) | (cj[k] >= I.n) |
                              (kLaneRows & ((v[k] >> si_shift) >= (uint32_t)(kWave / D))));
        }
        if (__ballot(bad) != 0) {
            if (bad)
                atomicAdd(I.cnt + kCntOverflow, 1ull);
            return;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (!live[k])
                continue;
            int res;
            if constexpr (Pol::kDot)
                res = pol.decide_dot(F[k], Q[k], ii[k], cj[k], tally, 0);
            else
                res = pol.decide(F[k], ii[k], cj[k], tally, 0);
            const uint32_t vk = v[k], ik = ii[k];
            pol.record(res, ik, cj[k],
                       [&]() {
                           return (uint64_t)ik * I.C +
                                  ((vk >> (B.bshift + 2)) & ((1u << B.tc_bits) - 1u));
                       },
                       (int)((vk >> B.bshift) & 3u), 0, tally);
        }
    };
    Win A, Bw;
    take(0);
    issue(A);
    if constexpr (kDepth == 2) {
        next(P);
        issue(Bw);
    }
    for (uint32_t k0 = 0; k0 < total; k0 += kDepth * P) {  // wave-uniform
        step(A, k0);
        if constexpr (kDepth == 2) {
            if (k0 + P >= total)
                break;
            step(Bw, k0 + P);
        }
    }
}

template <int D, bool kBuf, bool kLaneRows, class Pol>
__device__ __forceinline__ void eval_all_lds(const Inst &I, const BucketGeom &B, Pol &pol,
                                             Tally &tally, float *blk,
                                             unsigned long long *s_item)
{
    const uint32_t rows = 1u << B.bshift;
    const uint64_t chunks = (B.ranges + kLdsChunkRanges - 1) / kLdsChunkRanges;
    const uint64_t items = chunks * B.NJ;
    // wave index and item in scalar registers (uniform to the compiler)
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (;;) {
        __syncthreads();  // the last item's LDS reads are done, s_item is free
        if (threadIdx.x == 0)
            *s_item = atomicAdd(B.queue, 1ull);
        __syncthreads();
        const unsigned long long got = *s_item;
        const uint64_t it =
            ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(got >> 32))
             << 32) |
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
        if (it >= items)
            break;  // uniform over the workgroup
        const uint64_t c = it / B.NJ;
        const uint32_t J = (uint32_t)(it - c * B.NJ);
        const uint32_t j0 = J << B.bshift;
        const uint32_t nr = min(rows, I.n - j0);
        for (uint32_t e = threadIdx.x; e < nr * (uint32_t)D; e += kLdsThreads) {
            const uint32_t r = e / (uint32_t)D;
            blk[e] = I.X[(int64_t)(j0 + r) * I.ld + (e - r * (uint32_t)D)];
        }
        __syncthreads();
        const uint64_t rlo = c * kLdsChunkRanges;
        const uint64_t rhi = min(B.ranges, rlo + kLdsChunkRanges);
        for (uint64_t r0 = rlo + (uint64_t)wave * kLdsTicketRanges; r0 < rhi;
             r0 += (uint64_t)kLdsWaves * kLdsTicketRanges) {
            const uint64_t left = rhi - r0;
            const uint32_t T = (uint32_t)(left < kLdsTicketRanges ? left : kLdsTicketRanges);
            eval_ticket_lds<D, kLdsWindows, kBuf, kLaneRows>(I, B, pol, r0, T, J, tally, blk);
        }
    }
}

template <int D, bool kBuf, bool kLaneRows, int kQ>
__global__ __launch_bounds__(kLdsThreads) void k_bkt_eval_lds(Inst I, BucketGeom B)
{
    extern __shared__ float lds_blk[];
    __shared__ unsigned long long s_item;
    if (!sample_ok(I, B))
        return;
    BucketPlainPolicy<kQ> pol;
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
    eval_all_lds<D, kBuf, kLaneRows>(I, B, pol, t, lds_blk, &s_item);
    commit_tally(t, I.cnt);
}

template <int D, bool kBuf, bool kLaneRows>
__global__ __launch_bounds__(kLdsThreads) void k_bkt_eval_lds_sweep(Inst I, BucketGeom B,
                                                                    SweepArgs S)
{
    extern __shared__ float lds_blk[];
    __shared__ unsigned long long s_item;
    __shared__ float s_lo[kSweepMaxK], s_hi[kSweepMaxK];
    __shared__ double s_e2[kSweepMaxK];
    if (!sample_ok(I, B))
        return;
    for (int k = threadIdx.x; k < S.K; k += blockDim.x) {
        s_lo[k] = S.c.lo[k];
        s_hi[k] = S.c.hi[k];
        s_e2[k] = S.c.e2[k];
    }
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
    eval_all_lds<D, kBuf, kLaneRows>(I, B, pol, t, lds_blk, &s_item);  // its first barrier orders s_*
    commit_tally(t, I.cnt);
}

// Whether the source rows of every generator range fit one element per lane
// (then the LDS form keeps a segment's source rows in lanes): a range of
// kRangeCalls calls starting at call c0 < C of its first point ends at most
// (C - 1 + kRangeCalls - 1) / C points later.
inline bool lane_rows_fit(const Inst &I)
{
    return (((uint64_t)I.C - 1 + kRangeCalls - 1) / I.C + 1) * (uint64_t)I.d <= (uint64_t)kWave;
}

// Compute units of the current device. The persistent kernels (the sample
// kernel and the LDS form, whose LDS leaves room for one workgroup per CU)
// launch one workgroup per unit.
unsigned compute_units();

// Calls fn.template operator()<D>() for the compile-time row length D = d
// (1 <= d <= kLdsMaxD).
template <class Fn>
hipError_t dispatch_small_d(int d, Fn &&fn)
{
    switch (d) {
    case 1: return fn.template operator()<1>();
    case 2: return fn.template operator()<2>();
    case 3: return fn.template operator()<3>();
    case 4: return fn.template operator()<4>();
    case 5: return fn.template operator()<5>();
    case 6: return fn.template operator()<6>();
    case 7: return fn.template operator()<7>();
    case 8: return fn.template operator()<8>();
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Host side of the evaluate launches.
// ---------------------------------------------------------------------------
// Rows are read through a buffer descriptor with 32-bit byte offsets formed
// by 24-bit multiplies when X spans less than 4 GB, the row index fits 24
// bits and the row stride in bytes fits 24 bits.
inline bool use_buffer(const Inst &I)
{
    const uint64_t bytes = (uint64_t)I.n * (uint64_t)I.ld * 4u;
    return bytes < ((uint64_t)1 << 32) - 4096 && I.n < (1u << 24) &&
           (uint64_t)I.ld * 4u < ((uint64_t)1 << 24);
}

inline unsigned eval_blocks(const BucketGeom &B)
{
    // 128 blocks of 4 waves per XCD (four per CU), a multiple of kXcds
    (void)B;
    return kXcds * 128;
}

// The geometry as the evaluate kernels take it: with the byte span of X for
// the buffer form.
inline BucketGeom eval_geom(const Inst &I, const BucketGeom &B)
{
    BucketGeom g = B;
    g.x_bytes = use_buffer(I) ? (uint32_t)((uint64_t)I.n * (uint64_t)I.ld * 4u) : 0u;
    return g;
}

// Evaluate launch for query kQ (the sample already generated), and for the
// sweep; each is instantiated in a translation unit of its own.
template <int kQ>
hipError_t launch_bucket_eval(const Inst &I, const BucketGeom &B, const PassAShape &sh,
                              hipStream_t st)
{
    if (B.lds) {
        const size_t lds = ((size_t)1 << B.bshift) * (size_t)I.d * sizeof(float);
        const bool buf = use_buffer(I), lr = lane_rows_fit(I);
        return dispatch_small_d(I.d, [&]<int D>() -> hipError_t {
#define SNG_LDS_LAUNCH(BUF, LR)                                                              \
    hipLaunchKernelGGL((k_bkt_eval_lds<D, BUF, LR, kQ>), dim3(compute_units()),             \
                       dim3(kLdsThreads), lds, st, I, B)
            if (buf && lr) SNG_LDS_LAUNCH(true, true);
            else if (buf) SNG_LDS_LAUNCH(true, false);
            else if (lr) SNG_LDS_LAUNCH(false, true);
            else SNG_LDS_LAUNCH(false, false);
#undef SNG_LDS_LAUNCH
            return hipGetLastError();
        });
    }
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t) -> hipError_t {
        if constexpr (Row::kPrefetch) {
            if (use_buffer(I))
                hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB, true, kQ>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B);
            else
                hipLaunchKernelGGL((k_bkt_eval_plain<Row, OB, false, kQ>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

extern template hipError_t launch_bucket_eval<kSimNone>(const Inst &, const BucketGeom &,
                                                         const PassAShape &, hipStream_t);
extern template hipError_t launch_bucket_eval<kSimDot>(const Inst &, const BucketGeom &,
                                                        const PassAShape &, hipStream_t);
extern template hipError_t launch_bucket_eval<kSimCos>(const Inst &, const BucketGeom &,
                                                        const PassAShape &, hipStream_t);

hipError_t launch_bucket_eval_sweep(const Inst &I, const SweepArgs &S, const BucketGeom &B,
                                    const PassAShape &sh, hipStream_t st);

}  // namespace sng
