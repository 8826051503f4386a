// Hyperparameter sweep of SNG-DBSCAN: every (eps_k, MinPts_p) pair of a grid
// from one sampled-distance pass. The graphs are nested in eps (a pair
// accepted at eps_k is accepted at every larger eps) and the core sets are
// nested in eps and in MinPts, which is what makes one pass enough:
//   pass      level code of every slot: the smallest k with D <= eps_k^2
//             (K if none), and per-point histograms of the codes, so that
//             deg_k[i] = sum of the histogram of i up to k;
//   levels    core level kc_p[i] = smallest k with deg_k[i] >= MinPts_p;
//   hook      a slot with code b joins i and j in the union-find of level
//             e = max(b, kc_p[i], kc_p[j]) (the first level at which it is a
//             core-core edge), and offers a core endpoint to a non-core one
//             at level max(b, kc_p[core]) while the other is still non-core;
//   propagate for k = 0..K-2, every core point of level k is joined with its
//             level-k root at level k+1, so level k+1 holds every edge of the
//             levels below it;
//   finalize  core labels are roots; a non-core point takes the prefix minimum
//             of the offers up to k and the root of that core point.
// labels[p][k] then equals the single run at (eps_k, MinPts_p).
#include "sng_hook.hpp"
#include "sng_pass_a.hpp"

namespace sng {

// Level decision of one slot. Thresholds live in LDS.
struct SweepPolicy {
    int out_deg = 0;  // 1: out-degrees (no partner-side count)
    uint32_t *hist;   // [n][K]
    uint32_t *codes;  // one word of four level codes per Philox call
    const float *lo;
    const float *hi;
    const double *e2;
    int K;
    float hi_max;
    uint32_t own = 0;  // codes of this lane's own call

    static constexpr bool kDot = false;
    __device__ __forceinline__ void begin_chunk() { own = 0x01010101u * (uint32_t)K; }
    __device__ __forceinline__ void flush_source(uint32_t, int) {}
    __device__ __forceinline__ int decide(float F, uint32_t, uint32_t, const float *rowi,
                                          const float *rowj, int d, Tally &t, int q)
    {
        if (!(F <= hi_max))
            return K;  // beyond every band (or NaN): rejected at every level
        int a = 0, b = K - 1;  // first k with F <= hi[k]
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (F <= hi[mid])
                b = mid;
            else
                a = mid + 1;
        }
        if (F <= lo[a])
            return a;  // surely accepted at a, surely rejected below a
        t.rechecked += (q == 0);
        const double D = sqdist_f64(rowi, rowj, d);
        int k = a;
        while (k < K && !(D <= e2[k]))
            ++k;
        return k;
    }
    __device__ __forceinline__ void record(int b, uint32_t i, uint32_t j, int q, int o, int w,
                                           Tally &t)
    {
        if (b < K && q == 0) {
            atomicAdd(hist + (uint64_t)i * K + b, 1u);
            if (!out_deg)
                atomicAdd(hist + (uint64_t)j * K + b, 1u);
            t.accepted += 1;
        }
        if (q == o)
            own = (own & ~(0xFFu << (8 * w))) | ((uint32_t)b << (8 * w));
    }
    __device__ __forceinline__ void end_chunk(uint64_t gchunk, int lane)
    {
        codes[gchunk * 64ull + (uint64_t)lane] = own;
    }
};

template <class Row, int OB>
__global__ __launch_bounds__(256) void k_sweep_pass(Inst I, SweepArgs S, uint32_t cpw,
                                                    uint32_t slice_floats)
{
    extern __shared__ float lds[];
    __shared__ float s_lo[kSweepMaxK], s_hi[kSweepMaxK];
    __shared__ double s_e2[kSweepMaxK];
    for (int k = threadIdx.x; k < S.K; k += blockDim.x) {
        s_lo[k] = S.c.lo[k];
        s_hi[k] = S.c.hi[k];
        s_e2[k] = S.c.e2[k];
    }
    __syncthreads();
    SweepPolicy pol;
    pol.hist = S.hist;
    pol.codes = S.codes;
    pol.lo = s_lo;
    pol.hi = s_hi;
    pol.e2 = s_e2;
    pol.K = S.K;
    pol.hi_max = S.c.hi[S.K - 1];
    pol.out_deg = I.out_deg;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t lo = wave * cpw;
    float *slice = lds + (threadIdx.x / kWave) * slice_floats;
    Tally t;
    if (lo < I.chunks)  // wave-uniform
        pass_a_range<Row, OB>(I, pol, lo, min(lo + cpw, I.chunks), slice, t);
    commit_tally(t, I.cnt);
}

__device__ __forceinline__ int32_t *level_labels(const SweepArgs &S, uint32_t n, int p, int k)
{
    return S.labels + ((uint64_t)p * S.K + (uint64_t)k) * n;
}

// Degrees per level, core levels per MinPts, and the initial label arrays
// (parent = self for points that are core at that level, "no offer" else).
__global__ __launch_bounds__(256) void k_sweep_levels(Inst I, SweepArgs S)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint8_t kc[kSweepMaxP];
        for (int p = 0; p < S.P; ++p)
            kc[p] = (uint8_t)S.K;
        uint64_t run = 0;
        auto level = [&](int k, uint32_t h) {
            run += h;
            if (S.degrees)
                S.degrees[(uint64_t)k * I.n + i] = (uint32_t)run;
            for (int p = 0; p < S.P; ++p)
                if (kc[p] == S.K && (int64_t)run >= (int64_t)S.c.min_pts[p])
                    kc[p] = (uint8_t)k;
        };
        if ((S.K & 3) == 0) {  // the row is 16-byte aligned: four levels per load
            const uint4 *h4 = reinterpret_cast<const uint4 *>(S.hist + i * S.K);
            uint4 nx = h4[0];
            for (int k = 0; k < S.K; k += 4) {
                const uint4 h = nx;
                if (k + 4 < S.K)
                    nx = h4[(k >> 2) + 1];
                level(k, h.x);
                level(k + 1, h.y);
                level(k + 2, h.z);
                level(k + 3, h.w);
            }
        } else {
            for (int k = 0; k < S.K; ++k)
                level(k, S.hist[i * S.K + k]);
        }
        for (int p = 0; p < S.P; ++p) {
            S.kc[(uint64_t)p * I.n + i] = kc[p];
            for (int k = 0; k < S.K; ++k)
                level_labels(S, I.n, p, k)[i] = (kc[p] <= k) ? (int32_t)i : kNoCore;
        }
    }
}

// Level hook with block-local compaction: a round scans kSweepHookCalls
// calls' level codes (eight calls per thread, coalesced), lists the slots
// with a level below K in LDS, then the block's threads take the (listed
// slot, MinPts) pairs one each and regenerate their partners. A round lists
// about 80 slots on the 500k x 32 sweep; one thread per slot walking all
// MinPts values in turn (and rounds of 1024 calls) left most threads idle
// while a few ran four union chains each (sweep 12.1 ms against 11.3).
// Entry: call offset in the round (11 bits) << 8 | Philox word << 6 | level.
constexpr uint32_t kSweepHookCalls = 2048;

__global__ __launch_bounds__(256) void k_sweep_hook(Inst I, SweepArgs S)
{
    __shared__ uint32_t list[4 * kSweepHookCalls];
    __shared__ uint32_t nlist;
    const uint32_t none = 0x01010101u * (uint32_t)S.K;
    for (uint64_t c0 = (uint64_t)blockIdx.x * kSweepHookCalls; c0 < I.calls;
         c0 += (uint64_t)gridDim.x * kSweepHookCalls) {  // block-uniform
        if (threadIdx.x == 0)
            nlist = 0;
        uint32_t words[kSweepHookCalls / 256];
        uint32_t n = 0;
#pragma unroll
        for (int r = 0; r < (int)(kSweepHookCalls / 256); ++r) {
            const uint64_t call = c0 + (uint64_t)r * 256u + threadIdx.x;
            words[r] = (call < I.calls) ? S.codes[call] : none;
#pragma unroll
            for (int w = 0; w < 4; ++w)
                n += ((words[r] >> (8 * w)) & 0xFFu) < (uint32_t)S.K;
        }
        // the barrier also publishes the reset count; a round without listed
        // slots is skipped (nothing reads the list)
        if (!__syncthreads_or(n != 0u))
            continue;
        uint32_t pos = list_reserve(n, &nlist);
#pragma unroll
        for (int r = 0; r < (int)(kSweepHookCalls / 256); ++r) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t b = (words[r] >> (8 * w)) & 0xFFu;
                if (b < (uint32_t)S.K)
                    list[pos++] = ((r * 256u + threadIdx.x) << 8) | ((uint32_t)w << 6) | b;
            }
        }
        __syncthreads();
        const uint32_t cnt = nlist;
        for (uint32_t e = threadIdx.x; e < cnt * (uint32_t)S.P; e += blockDim.x) {
            const int p = (int)(e / cnt);
            const uint32_t v = list[e - (uint32_t)p * cnt];
            const uint64_t call = c0 + (v >> 8);
            const int w = (int)((v >> 6) & 3u);
            const int b = (int)(v & 63u);
            const uint32_t i = (uint32_t)div_exact64(call, I.C, I.inv_C);
            const uint32_t c = (uint32_t)(call - (uint64_t)i * I.C);
            const Words4 W = philox10(c, i, I.key0, I.key1);
            const uint32_t j = mod_exact(W.w[w], I.n, I.inv_n);
            const int ki = S.kc[(uint64_t)p * I.n + i];
            const int kj = S.kc[(uint64_t)p * I.n + j];
            const int lev = max(b, max(ki, kj));
            if (lev < S.K)
                uf_unite(level_labels(S, I.n, p, lev), (int32_t)i, (int32_t)j);
            const int ei = max(b, ki);  // i is a core neighbour of j from ei on
            if (ei < kj)
                atomicMin(level_labels(S, I.n, p, ei) + j, (int32_t)i);
            const int ej = max(b, kj);
            if (ej < ki)
                atomicMin(level_labels(S, I.n, p, ej) + i, (int32_t)j);
        }
        __syncthreads();  // the next round reuses the list
    }
}

// Level k -> k+1 in two launches. Level k is final. k_sweep_stars writes
// each core point's level-k root into its level-k entry (level k is then
// compressed) and into its level-(k+1) entry, so level k+1 starts from level
// k's components with one plain store per point. The level-(k+1) links those
// stores replace, unions born at k+1, go to `link`; k_sweep_relink joins them
// again (the links of a level run between few large components, hence the
// verified hook). Points that only become core at k+1 keep their links in
// place. One union per core point instead (every point with its level-k
// root) made the threads of a large component race compare-and-swaps on one
// shared root.
__global__ __launch_bounds__(256) void k_sweep_stars(Inst I, SweepArgs S, int k)
{
    const uint64_t total = (uint64_t)S.P * I.n;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const int p = (int)(u / I.n);
        const uint32_t x = (uint32_t)(u - (uint64_t)p * I.n);
        if (S.kc[u] > k)
            continue;
        // entries of level k only move to their roots here, so a walk
        // through cached (possibly older) parents still ends at the root
        int32_t *L0 = level_labels(S, I.n, p, k);
        int32_t r = (int32_t)x, q = uf_ld(L0 + x);
        while (q != r) {
            r = q;
            q = uf_ld(L0 + r);
        }
        uf_st(L0 + x, r);
        int32_t *L1 = level_labels(S, I.n, p, k + 1);
        S.link[u] = L1[x];
        L1[x] = r;
    }
}

__global__ __launch_bounds__(256) void k_sweep_relink(Inst I, SweepArgs S, int k)
{
    const uint64_t total = (uint64_t)S.P * I.n;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const int p = (int)(u / I.n);
        const uint32_t x = (uint32_t)(u - (uint64_t)p * I.n);
        if (S.kc[u] > k)
            continue;
        const int32_t e = S.link[u];
        if (e != (int32_t)x)
            uf_unite_verified(level_labels(S, I.n, p, k + 1), (int32_t)x, e);
    }
}

// The last level's roots (the levels below were compressed by k_sweep_stars).
__global__ __launch_bounds__(256) void k_sweep_compress(Inst I, SweepArgs S)
{
    const uint64_t total = (uint64_t)S.P * I.n;
    const int k = S.K - 1;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const int p = (int)(u / I.n);
        const uint32_t x = (uint32_t)(u - (uint64_t)p * I.n);
        if (S.kc[u] <= k) {
            int32_t *L = level_labels(S, I.n, p, k);
            st_relaxed(L + x, uf_root(L, (int32_t)x));
        }
    }
}

__global__ __launch_bounds__(256) void k_sweep_borders(Inst I, SweepArgs S)
{
    const uint64_t total = (uint64_t)S.P * I.n;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const int p = (int)(u / I.n);
        const uint32_t x = (uint32_t)(u - (uint64_t)p * I.n);
        const int kend = min((int)S.kc[u], S.K);
        int32_t best = kNoCore;
        // eight levels at a time: their offers, then their labels, are loaded
        // together (x is not core below kend, so no thread reads L[x] there)
        for (int k0 = 0; k0 < kend; k0 += 8) {
            int32_t off[8], bst[8], lab[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                off[t] = (k0 + t < kend) ? level_labels(S, I.n, p, k0 + t)[x] : kNoCore;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                best = min(best, off[t]);
                bst[t] = best;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
                lab[t] = (k0 + t < kend && bst[t] != kNoCore)
                             ? level_labels(S, I.n, p, k0 + t)[bst[t]]
                             : -1;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (k0 + t < kend)
                    level_labels(S, I.n, p, k0 + t)[x] = lab[t];
        }
    }
}

static unsigned sweep_grid(uint64_t items)
{
    const uint64_t g = (items + 255) / 256;
    return (unsigned)(g == 0 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_sweep(const Inst &I, const SweepArgs &S, const PassAShape &sh,
                        const BucketGeom *B, hipStream_t st)
{
    hipError_t e;
    if (I.n == 0)
        return hipSuccess;
    if (I.m > 0 && I.chunks > 0 && B) {
        e = launch_fill_u32(S.codes, I.chunks * 64, 0x01010101u * (uint32_t)S.K, st);
        if (e != hipSuccess)
            return e;
        e = launch_bucket_sweep(I, S, *B, sh, st);
        if (e != hipSuccess)
            return e;
    } else if (I.m > 0 && I.chunks > 0) {
        const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
        e = dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t slice) -> hipError_t {
            const uint64_t waves = (I.chunks + sh.chunks_per_wave - 1) / sh.chunks_per_wave;
            const uint64_t blocks = (waves + sh.waves_per_block - 1) / sh.waves_per_block;
            if (blocks > 0x7FFFFFFFull)
                return hipErrorInvalidValue;
            const size_t lds = (size_t)slice * sizeof(float) * sh.waves_per_block;
            hipLaunchKernelGGL((k_sweep_pass<Row, OB>), dim3((unsigned)blocks),
                               dim3(64 * sh.waves_per_block), lds, st, I, S,
                               (uint32_t)sh.chunks_per_wave, slice);
            return hipGetLastError();
        });
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_sweep_levels, dim3(sweep_grid(I.n)), dim3(256), 0, st, I, S);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (I.m > 0) {
        hipLaunchKernelGGL(k_sweep_hook, dim3(sweep_grid(I.calls)), dim3(256), 0, st, I, S);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const unsigned grid = sweep_grid((uint64_t)S.P * I.n);
    for (int k = 0; k + 1 < S.K; ++k) {
        hipLaunchKernelGGL(k_sweep_stars, dim3(grid), dim3(256), 0, st, I, S, k);
        hipLaunchKernelGGL(k_sweep_relink, dim3(grid), dim3(256), 0, st, I, S, k);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_sweep_compress, dim3(grid), dim3(256), 0, st, I, S);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sweep_borders, dim3(sweep_grid((uint64_t)S.P * I.n)), dim3(256), 0, st,
                       I, S);
    return hipGetLastError();
}

}  // namespace sng
