// C ABI of libsng.so: argument validation, workspace layout and the launch
// sequence of each entry point (declarations and contracts in sng.h).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sng.h"
#include "sng_internal.hpp"

using namespace sng;

namespace {

constexpr size_t kHeaderBytes = 4096;  // counters of one instance
constexpr size_t kInstHeader = 256;    // counters of instance k sit at k*256 in a batch
constexpr size_t kAlign = 256;
constexpr int64_t kMaxN = 2147483647LL;
constexpr int64_t kMaxM = 2147483648LL;  // t/4 and 4*C stay in 32 bits

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count)
    {
        T *p = (T *)(base + off);
        off = align_up(off + count * sizeof(T));
        return p;
    }
};

int m_from_s(double s, int64_t n, int64_t *m)
{
    if (!(s >= 0.0) || isinf(s) || n < 0)
        return SNG_EINVAL;
    const double v = ceil(s * (double)n);
    if (v > (double)kMaxM)
        return SNG_ERANGE;
    *m = (int64_t)v;
    return SNG_OK;
}

int check_points(const void *X, int64_t n, int32_t d, int64_t ld)
{
    if (n < 0 || d < 1 || ld < d)
        return SNG_EINVAL;
    if (n > kMaxN)
        return SNG_ERANGE;
    if (n > 0 && (!X || ((uintptr_t)X & 3u)))
        return SNG_EINVAL;
    if (ld > (int64_t)1 << 40)
        return SNG_ERANGE;
    return SNG_OK;
}

int check_eps(double eps)
{
    return (eps >= 0.0 && !isinf(eps)) ? SNG_OK : SNG_EINVAL;
}

struct Sizes {
    uint64_t C = 0, calls = 0, chunks = 0;
};

Sizes sizes_for(int64_t n, int64_t m)
{
    Sizes z;
    z.C = (uint64_t)((m + 3) / 4);
    z.calls = (uint64_t)n * z.C;
    z.chunks = (z.calls + 63) / 64;
    return z;
}

size_t plain_ws_bytes(int64_t n, int64_t m)
{
    const Sizes z = sizes_for(n, m);
    size_t b = kHeaderBytes;
    b = align_up(b + (size_t)n * 4);     // degrees
    b = align_up(b + (size_t)n);         // core flags
    b = align_up(b + z.chunks * 8 * 4);  // accept bits
    return b;
}

// The simple-graph degree mode adds the hash table of accepted pairs, sized
// for every slot accepted (2^simple_table_log2 u64 entries), at most
// 2^kSimpleMaxLog2 entries (512 GB, more than a GPU holds).
constexpr uint32_t kSimpleMaxLog2 = 36;

size_t simple_ws_bytes(int64_t n, int64_t m)
{
    return align_up(((size_t)1 << simple_table_log2(n, m)) * sizeof(unsigned long long));
}

// SNG_ERANGE when the simple-graph table of (n, m) would exceed the cap.
int check_simple(const sng_config *cfg, int64_t n, int64_t m)
{
    if (cfg && cfg->simple_graph && simple_table_log2(n, m) > kSimpleMaxLog2)
        return SNG_ERANGE;
    return SNG_OK;
}

// The cosine query adds a unit-length copy of the rows; the dot product
// nothing.
size_t sim_rows_floats(int64_t n, int32_t d, int32_t kind)
{
    return kind == SNG_SIM_COSINE ? (size_t)n * (size_t)unit_copy_ld(d) : 0u;
}

size_t sim_ws_bytes(int64_t n, int32_t d, int64_t m, int32_t kind)
{
    return align_up(plain_ws_bytes(n, m) + sim_rows_floats(n, d, kind) * sizeof(float));
}

// The mixed-precision pass adds per-row statistics and a queue of undecided
// slots large enough for every slot, so it can never overflow.
size_t lowp_ws_bytes(int64_t n, int64_t m)
{
    size_t b = plain_ws_bytes(n, m);
    b = align_up(b + (size_t)n * 4 * sizeof(double));
    b = align_up(b + (size_t)n * (size_t)m * sizeof(uint64_t));
    return b;
}

inline int hip_rc(hipError_t e) { return e == hipSuccess ? SNG_OK : SNG_EHIP; }

#define SNG_TRY(expr)                       \
    do {                                    \
        const hipError_t e_ = (expr);       \
        if (e_ != hipSuccess)               \
            return SNG_EHIP;                \
    } while (0)

// Fills the descriptor of one plain instance whose buffers are already carved.
Inst make_inst(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
               uint64_t seed, int32_t min_pts)
{
    Inst I;
    memset(&I, 0, sizeof(I));
    const Sizes z = sizes_for(n, m);
    I.X = X;
    I.ld = ld;
    I.n = (uint32_t)n;
    I.d = d;
    I.m = (uint32_t)m;
    I.C = (uint32_t)z.C;
    I.key0 = (uint32_t)(seed & 0xFFFFFFFFull);
    I.key1 = (uint32_t)(seed >> 32);
    I.inv_n = n > 0 ? 1.0 / (double)n : 0.0;
    I.inv_nf = (n >= 1024 && n <= ((int64_t)1 << 30)) ? (float)(1.0 / (double)n) : 0.0f;
    I.inv_C = z.C > 0 ? 1.0 / (double)z.C : 0.0;
    I.eps2 = eps * eps;
    band_fp32(I.eps2, d, &I.lo, &I.hi, &I.band);
    I.calls = z.calls;
    I.chunks = z.chunks;
    I.chunk0 = 0;
    I.min_pts = min_pts;
    return I;
}

// bucketed: the partner-block schedule, whose evaluate kernel keeps the
// source row of every record in flight too; it defaults to 4 records in
// flight per group (fewer registers, twice the waves per SIMD).
PassAShape shape_for(const Inst &I, const sng_config *cfg, bool bucketed = false)
{
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    int prefetch = cfg ? cfg->prefetch : 0;
    if (bucketed && prefetch == 0)
        prefetch = 4;
    // Direct gathers default to eight chunks per wavefront, fewer when that
    // would leave fewer than 4096 wavefronts (small instances: the 10k x 2
    // call has 3907 chunks; one chunk per wave takes the call from 78 to
    // 73 us).
    int cpw = cfg ? cfg->chunks_per_wave : 0;
    if (cpw == 0 && !bucketed) {
        const uint64_t per = I.chunks / 4096;
        cpw = per >= 8 ? 8 : (per >= 1 ? (int)per : 1);
    }
    return resolve_shape(I.d, vec_ok, cfg ? cfg->lanes_per_pair : 0, cpw,
                         cfg ? cfg->stage_lds : 0, prefetch);
}

int check_cfg(const sng_config *cfg)
{
    if (!cfg)
        return SNG_OK;
    const int g = cfg->lanes_per_pair;
    if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64)
        return SNG_EINVAL;
    if (cfg->chunks_per_wave < 0 || cfg->chunks_per_wave > 4096)
        return SNG_EINVAL;
    if (cfg->prefetch != 0 && cfg->prefetch != 4 && cfg->prefetch != 8 && cfg->prefetch != 16)
        return SNG_EINVAL;
    if (cfg->schedule < 0 || cfg->schedule > 2)
        return SNG_EINVAL;
    if (cfg->reuse_sample != 0 && cfg->reuse_sample != 1)
        return SNG_EINVAL;
    if (cfg->reuse_sample && (cfg->schedule == 1 || cfg->stage_lds))
        return SNG_EINVAL;  // a stored sample is evaluated by the partner-block schedule only
    if (cfg->out_degree != 0 && cfg->out_degree != 1)
        return SNG_EINVAL;
    if (cfg->simple_graph != 0 && cfg->simple_graph != 1)
        return SNG_EINVAL;
    if (cfg->simple_graph && (cfg->out_degree || cfg->reuse_sample))
        return SNG_EINVAL;  // one degree mode at a time; the table moves the sample
    const int w = cfg->mfma_waves, k = cfg->mfma_ksteps, h = cfg->hook_blocks;
    if (w != 0 && w != 1 && w != 2 && w != 4)
        return SNG_EINVAL;
    if (k != 0 && k != 4 && k != 8 && k != 16)
        return SNG_EINVAL;
    if (h != 0 && (h < 256 || h > 65536))
        return SNG_EINVAL;
    return SNG_OK;
}

// The counters of a call (threads 0..kCntNum-1 of one block).
__device__ __forceinline__ void write_header(unsigned long long *cnt, unsigned long long slots,
                                             double band, int keep_sample)
{
    const int t = threadIdx.x;
    if (t < kCntNum || (t > kCntNum && t < kFltEnd))
        cnt[t] = (t == kCntSlots) ? slots : 0ull;
    if (t == 0)
        ((double *)(cnt + kCntNum))[0] = band;
    if (!keep_sample && t < 2)
        cnt[kSampleHdr + t] = 0ull;  // this layout holds no partner-block sample
}

__global__ void k_header(unsigned long long *cnt, unsigned long long slots, double band,
                         int keep_sample)
{
    write_header(cnt, slots, band, keep_sample);
}

// The header of init_header plus deg[0..n) = 0, in one launch.
__global__ void k_init_call(unsigned long long *cnt, unsigned long long slots, double band,
                            int keep_sample, uint32_t *deg, uint64_t n)
{
    if (blockIdx.x == 0)
        write_header(cnt, slots, band, keep_sample);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        deg[i] = 0u;
}

// Counters of a call. keep_sample: the call uses the plain layout, so a
// partner-block sample stored by an earlier call stays valid; every other
// layout overwrites the record area and clears the sample's tag.
hipError_t init_header(unsigned long long *cnt, uint64_t slots, double band, hipStream_t st,
                       bool keep_sample = false)
{
    hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, st, cnt, (unsigned long long)slots, band,
                       keep_sample ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Autotune cache: the fastest configuration found by sng_autotune for a
// shape class, used by calls that pass no configuration of their own.
// ---------------------------------------------------------------------------
constexpr int kPreferPartner = 3;  // internal schedule: partner blocks when they fit, else direct

// Forms with tuned shapes of their own (the key's first field).
enum TuneForm : int { kFormPlain = 0, kFormBf16 = 1, kFormFp16 = 2, kFormBatch = 3 };

struct TuneKey {
    int form, d, vec, lg_n, lg_m;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(form, d, vec, lg_n, lg_m) <
               std::tie(o.form, o.d, o.vec, o.lg_n, o.lg_m);
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, sng_config> g_tune;

// The cache file: this header line, then one entry per line.
const char *const kTuneFileHeader = "sng-autotune 1";
constexpr int kConfigFields = (int)(sizeof(sng_config) / sizeof(int32_t));
static_assert(sizeof(sng_config) == 11 * sizeof(int32_t), "the file lists every field");

int ceil_log2(uint64_t v)
{
    int r = 0;
    while (r < 63 && ((uint64_t)1 << r) < v)
        ++r;
    return r;
}

TuneKey tune_key(const float *X, int32_t d, int64_t ld, int64_t n, int64_t m,
                 int form = kFormPlain)
{
    const int vec = ((uintptr_t)X % 16 == 0) && (ld % 4 == 0);
    return TuneKey{form, d, vec, ceil_log2((uint64_t)n), ceil_log2((uint64_t)m)};
}

// No launch shape chosen by the caller (the degree modes are not launch choices).
bool is_default_cfg(const sng_config *cfg)
{
    return !cfg || (cfg->lanes_per_pair == 0 && cfg->chunks_per_wave == 0 && cfg->stage_lds == 0 &&
                    cfg->prefetch == 0 && cfg->schedule == 0 && cfg->reuse_sample == 0 &&
                    cfg->mfma_waves == 0 && cfg->mfma_ksteps == 0 && cfg->hook_blocks == 0);
}

// The cached configuration of `key`, if any.
bool tuned_entry(const TuneKey &key, sng_config *out)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it == g_tune.end())
        return false;
    *out = it->second;
    return true;
}

// The configuration a call runs with: the caller's own, or for a call without
// one the tuned configuration of its shape class if there is one. A tuned
// partner-block schedule becomes a preference, so a workspace sized for
// direct gathers still works.
const sng_config *effective_cfg(const Inst &I, const sng_config *cfg, sng_config *buf,
                                int form = kFormPlain)
{
    if (!is_default_cfg(cfg))
        return cfg;
    if (!tuned_entry(tune_key(I.X, I.d, I.ld, I.n, I.m, form), buf))
        return cfg;
    if (buf->schedule == 2)
        buf->schedule = kPreferPartner;
    buf->out_degree = cfg ? cfg->out_degree : 0;
    buf->simple_graph = cfg ? cfg->simple_graph : 0;
    return buf;
}

// Chooses the schedule of the sampled-distance pass: the partner-block
// schedule when it applies, the caller allows it and the workspace holds its
// records (carved after `used` bytes); otherwise direct gathers.
int pick_bucket(const Inst &I, const sng_config *cfg, void *workspace, size_t ws_bytes,
                size_t used, BucketGeom *B, bool *use, uint32_t layout = kLayoutPlain)
{
    *use = false;
    if (I.m == 0 || I.n == 0)
        return SNG_OK;  // no sampled-distance pass to schedule
    const int sched = cfg ? cfg->schedule : 0;
    const bool forced = sched == 2 || (cfg && cfg->reuse_sample);
    if (sched == 1 || (cfg && cfg->stage_lds))
        return forced ? SNG_EINVAL : SNG_OK;
    if (!bucket_geometry(I.n, I.d, I.m, forced || sched == kPreferPartner, B))
        return forced ? SNG_ENOTIMPL : SNG_OK;
    if (align_up(used + bucket_bytes(*B)) > ws_bytes)
        return forced ? SNG_EWORKSPACE : SNG_OK;
    Carve cv((char *)workspace + used);
    B->rec = cv.take<uint32_t>(B->ranges * B->region);
    B->seg = cv.take<uint32_t>(B->ranges * B->NJ * 2);
    B->start = cv.take<uint32_t>(B->ranges * 2);
    B->queue = cv.take<unsigned long long>(kXcds);
    B->hdr = I.cnt + kSampleHdr;
    // the block size and the record format (LDS or not) both fix the records
    B->tag = sample_tag(I.n, I.m, (uint64_t)I.key0 | ((uint64_t)I.key1 << 32),
                        B->bshift | (B->lds << 8), layout);
    *use = true;
    return SNG_OK;
}

// Per-row data of a similarity instance (see launch_similarity_rows).
struct SimRows {
    float *unit = nullptr;  // cosine: unit-length copy of the rows
};

// The simple-graph table of a call, null when the mode is off.
struct SimpleTable {
    unsigned long long *table = nullptr;
    uint32_t max_log2 = 0;
};

// Carves the simple-graph table when cfg asks for the mode.
SimpleTable carve_simple(Carve &cv, const sng_config *cfg, int64_t n, int64_t m)
{
    SimpleTable s;
    if (cfg && cfg->simple_graph) {
        s.max_log2 = simple_table_log2(n, m);
        s.table = cv.take<unsigned long long>((size_t)1 << s.max_log2);
    }
    return s;
}

// Pass (a) plus post-processing for one carved instance. sim: the per-row
// arrays of a similarity instance (written first), else null. simple: the
// table of the simple-graph degree mode (table null: multigraph degrees).
int run_plain(Inst &I, const sng_config *cfg, bool labels_wanted, const BucketGeom *B,
              hipStream_t st, const SimRows *sim = nullptr, const SimpleTable &simple = {})
{
    // only the plain layout keeps a stored partner-block sample valid
    {
        const uint64_t blocks = ((uint64_t)I.n + 255) / 256;
        hipLaunchKernelGGL(k_init_call, dim3(blocks == 0 ? 1 : (blocks > 4096 ? 4096 : blocks)),
                           dim3(256), 0, st, I.cnt, (unsigned long long)I.n * I.m, I.band,
                           (sim == nullptr && simple.table == nullptr) ? 1 : 0, I.deg,
                           (uint64_t)I.n);
        SNG_TRY(hipGetLastError());
    }
    if (sim && I.m > 0)
        SNG_TRY(launch_similarity_rows(I, sim->unit, st));
    if (I.m > 0 && B) {
        SNG_TRY(launch_fill_u32(I.mask, I.chunks * 8, 0u, st));
        SNG_TRY(launch_bucket_plain(I, *B, shape_for(I, cfg, true),
                                    cfg && cfg->reuse_sample, st));
    } else if (I.m > 0) {
        SNG_TRY(launch_pass_a(I, shape_for(I, cfg), st));
    }
    if (simple.table)
        SNG_TRY(launch_simple_degrees(I, simple.table, simple.max_log2,
                                      reinterpret_cast<uint32_t *>(I.cnt + kSimpleHdr), st));
    if (!labels_wanted)
        return SNG_OK;
    SNG_TRY(launch_core_init(I, st));
    if (I.m > 0)
        SNG_TRY(launch_hook_mask(I, st, cfg ? (unsigned)cfg->hook_blocks : 0u));
    SNG_TRY(launch_finalize(I, st));
    return SNG_OK;
}

// Mean ms of `trials` calls of run() on st after one warm-up call (HIP
// events; synchronises st). run returns a status; the first failure is
// returned as is.
template <class Run>
int time_calls(hipStream_t st, int trials, Run &&run, float *ms)
{
    int rc = run();
    if (rc != SNG_OK)
        return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SNG_EHIP;
    }
    if (hipEventRecord(e0, st) != hipSuccess)
        rc = SNG_EHIP;
    for (int k = 0; k < trials && rc == SNG_OK; ++k)
        rc = run();
    float t = 0.0f;
    if (rc == SNG_OK && (hipEventRecord(e1, st) != hipSuccess ||
                         hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = SNG_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / (float)trials;
    return rc;
}

// Times every candidate with run(config) (a candidate that fails with
// SNG_EINVAL or SNG_ENOTIMPL is skipped as not applicable) and keeps the
// fastest in *best, its mean time in *best_ms and the number timed in
// *tried (both may be null).
template <class Run>
int tune_candidates(const std::vector<sng_config> &cand, hipStream_t st, int trials, Run &&run,
                    sng_config *best, float *best_ms, int32_t *tried)
{
    float best_t = -1.0f;
    int n_tried = 0;
    for (const sng_config &c : cand) {
        float ms = 0.0f;
        const int rc = time_calls(st, trials, [&]() { return run(c); }, &ms);
        if (rc == SNG_EINVAL || rc == SNG_ENOTIMPL)
            continue;
        if (rc != SNG_OK)
            return rc;
        ++n_tried;
        if (best_t < 0.0f || ms < best_t) {
            best_t = ms;
            *best = c;
        }
    }
    if (tried) *tried = n_tried;
    if (best_t < 0.0f)
        return SNG_ENOTIMPL;
    if (best_ms) *best_ms = best_t;
    return SNG_OK;
}

}  // namespace

extern "C" {

const char *sng_status_string(int status)
{
    switch (status) {
    case SNG_OK: return "ok";
    case SNG_EINVAL: return "invalid argument";
    case SNG_ERANGE: return "size out of range";
    case SNG_EWORKSPACE: return "workspace missing or too small";
    case SNG_EHIP: return "HIP runtime error";
    case SNG_EOVERFLOW: return "device queue overflow";
    case SNG_ENOTIMPL: return "not implemented for these arguments";
    case SNG_EIO: return "file could not be opened, read or written";
    default: return "unknown status";
    }
}

int sng_samples_per_point(double s, int64_t n, int64_t *m)
{
    if (!m)
        return SNG_EINVAL;
    return m_from_s(s, n, m);
}

int sng_workspace_size(int64_t n, int32_t d, int64_t m, int32_t prec, size_t *bytes)
{
    if (!bytes || n < 0 || d < 1 || m < 0)
        return SNG_EINVAL;
    if (n > kMaxN || m > kMaxM)
        return SNG_ERANGE;
    const bool direct_only = (prec & SNG_WS_DIRECT) != 0;
    const bool simple = (prec & SNG_WS_SIMPLE_GRAPH) != 0;
    prec &= ~(SNG_WS_DIRECT | SNG_WS_SIMPLE_GRAPH);
    if (prec != SNG_FP32 && prec != SNG_BF16 && prec != SNG_FP16)
        return SNG_EINVAL;
    if (prec != SNG_FP32) {
        if (simple)
            return SNG_EINVAL;  // the mixed form has no simple-graph mode
        *bytes = lowp_ws_bytes(n, m);
        return SNG_OK;
    }
    if (simple && simple_table_log2(n, m) > kSimpleMaxLog2)
        return SNG_ERANGE;
    size_t b = plain_ws_bytes(n, m) + (simple ? simple_ws_bytes(n, m) : 0);
    BucketGeom g;
    if (!direct_only && bucket_geometry(n, d, m, true, &g))
        b = align_up(b + bucket_bytes(g));
    *bytes = b;
    return SNG_OK;
}

int sng_degrees(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                uint64_t seed, uint32_t *degrees, void *workspace, size_t ws_bytes,
                const sng_config *cfg, void *stream)
{
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if ((rc = check_eps(eps))) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if (m < 0) return SNG_EINVAL;
    if (m > kMaxM) return SNG_ERANGE;
    if (n > 0 && !degrees) return SNG_EINVAL;
    if ((rc = check_simple(cfg, n, m))) return rc;
    const size_t need =
        plain_ws_bytes(n, m) + (cfg && cfg->simple_graph ? simple_ws_bytes(n, m) : 0);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, eps, seed, 0);
    I.out_deg = (cfg && cfg->out_degree) ? 1 : 0;
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    (void)cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    I.mask = cv.take<uint32_t>(sizes_for(n, m).chunks * 8);
    const SimpleTable simple = carve_simple(cv, cfg, n, m);
    I.deg = degrees;
    I.labels = nullptr;
    sng_config tuned;
    cfg = effective_cfg(I, cfg, &tuned);
    BucketGeom B;
    bool use = false;
    const uint32_t layout = simple.table ? kLayoutPlain | kLayoutSimpleTable : kLayoutPlain;
    if ((rc = pick_bucket(I, cfg, workspace, ws_bytes, cv.off, &B, &use, layout))) return rc;
    return run_plain(I, cfg, false, use ? &B : nullptr, st, nullptr, simple);
}

int sng_sample(int64_t n, int32_t d, int64_t m, uint64_t seed, void *workspace, size_t ws_bytes,
               void *stream)
{
    if (n < 0 || d < 1 || m < 0)
        return SNG_EINVAL;
    if (n > kMaxN || m > kMaxM)
        return SNG_ERANGE;
    const size_t need = plain_ws_bytes(n, m);
    if (!workspace || ws_bytes < need)
        return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(nullptr, n, d, d, m, 0.0, seed, 0);
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    (void)cv.take<uint32_t>((size_t)n);
    (void)cv.take<uint8_t>((size_t)n);
    (void)cv.take<uint32_t>(sizes_for(n, m).chunks * 8);
    if (n == 0 || m == 0)
        return SNG_OK;  // an empty sample: sng_degrees has nothing to evaluate
    sng_config force;
    memset(&force, 0, sizeof(force));
    force.schedule = 2;
    BucketGeom B;
    bool use = false;
    int rc = pick_bucket(I, &force, workspace, ws_bytes, cv.off, &B, &use);
    if (rc)
        return rc;
    SNG_TRY(launch_bucket_generate(I, B, st));
    return SNG_OK;
}

int sng_autotune(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                 uint64_t seed, void *workspace, size_t ws_bytes, int32_t trials,
                 sng_config *best, float *best_ms, int32_t *tried, void *stream)
{
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if ((rc = check_eps(eps))) return rc;
    if (m < 0 || !best || trials < 1 || trials > 1000) return SNG_EINVAL;
    if (m > kMaxM) return SNG_ERANGE;
    const size_t need = plain_ws_bytes(n, m);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    memset(best, 0, sizeof(*best));
    if (best_ms) *best_ms = 0.0f;
    if (tried) *tried = 0;
    if (n == 0 || m == 0)
        return SNG_OK;  // no sampled-distance pass to tune
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, eps, seed, 0);
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    I.deg = cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    I.mask = cv.take<uint32_t>(sizes_for(n, m).chunks * 8);
    I.labels = nullptr;

    // Candidates: lanes per pair around the default, rows in flight, chunks
    // per wave (direct), LDS staging for wide rows, and both schedules; the
    // shapes that resolve to the same launch are tried once.
    const bool vec_ok = ((uintptr_t)X % 16 == 0) && (ld % 4 == 0);
    const int g0 = resolve_shape(d, vec_ok, 0, 0, 0, 0).lanes;
    std::vector<sng_config> cand;
    std::vector<std::tuple<int, int, int, int, int>> seen;
    auto add = [&](int sched, int lanes, int cpw, int lds, int pf) {
        const PassAShape s = resolve_shape(d, vec_ok, lanes, cpw, lds, pf);
        const auto key = std::make_tuple(sched, s.lanes, sched == 2 ? 0 : s.chunks_per_wave,
                                         s.stage_lds, s.owners_per_batch);
        for (const auto &k : seen)
            if (k == key) return;
        seen.push_back(key);
        sng_config c;
        memset(&c, 0, sizeof(c));
        c.schedule = sched;
        c.lanes_per_pair = s.lanes;
        c.chunks_per_wave = sched == 2 ? 0 : s.chunks_per_wave;
        c.stage_lds = s.stage_lds;
        c.prefetch = 4 * s.owners_per_batch;
        cand.push_back(c);
    };
    for (int g : {g0, g0 / 2, g0 * 2}) {
        if (g < 1 || g > 64) continue;
        for (int pf : {4, 8, 16}) {
            for (int cpw : {8, 16})
                add(1, g, cpw, 0, pf);
            add(2, g, 0, 0, pf);
        }
    }
    if (d >= 256 && d <= 4096)
        add(1, 64, 8, 1, 4);

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SNG_EHIP;
    }
    float best_t = -1.0f;
    int n_tried = 0;
    rc = SNG_OK;
    for (const sng_config &c : cand) {
        BucketGeom B;
        bool use = false;
        if (pick_bucket(I, &c, workspace, ws_bytes, cv.off, &B, &use) != SNG_OK)
            continue;  // this schedule does not apply, or the workspace lacks its records
        const BucketGeom *bp = use ? &B : nullptr;
        if ((rc = run_plain(I, &c, false, bp, st)) != SNG_OK)  // warm-up
            break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = SNG_EHIP; break; }
        for (int k = 0; k < trials && rc == SNG_OK; ++k)
            rc = run_plain(I, &c, false, bp, st);
        if (rc != SNG_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = SNG_EHIP;
            break;
        }
        ms /= (float)trials;
        ++n_tried;
        if (best_t < 0.0f || ms < best_t) {
            best_t = ms;
            *best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SNG_OK)
        return rc;
    if (tried) *tried = n_tried;
    if (best_t < 0.0f)
        return SNG_ENOTIMPL;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    sng_config &e = g_tune[tune_key(X, d, ld, n, m)];
    const int32_t hook = e.hook_blocks;  // tuned separately (sng_autotune_hook)
    e = *best;
    e.hook_blocks = hook;
    return SNG_OK;
}

int sng_autotune_lookup(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                        sng_config *out)
{
    if (!out || n < 0 || d < 1 || ld < d || m < 0)
        return SNG_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(tune_key(X, d, ld, n, m));
    if (it == g_tune.end())
        return SNG_ENOTIMPL;
    *out = it->second;
    return SNG_OK;
}

int sng_autotune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    return SNG_OK;
}

int sng_autotune_save(const char *path)
{
    if (!path)
        return SNG_EINVAL;
    std::ostringstream out;
    out << kTuneFileHeader << "\n";
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const auto &kv : g_tune) {
            const TuneKey &k = kv.first;
            const int32_t *f = reinterpret_cast<const int32_t *>(&kv.second);
            out << k.form << ' ' << k.d << ' ' << k.vec << ' ' << k.lg_n << ' ' << k.lg_m;
            for (int i = 0; i < kConfigFields; ++i)
                out << ' ' << f[i];
            out << "\n";
        }
    }
    FILE *fp = fopen(path, "w");
    if (!fp)
        return SNG_EIO;
    const std::string text = out.str();
    const bool ok = fwrite(text.data(), 1, text.size(), fp) == text.size();
    return (fclose(fp) == 0 && ok) ? SNG_OK : SNG_EIO;
}

int sng_autotune_load(const char *path)
{
    if (!path)
        return SNG_EINVAL;
    FILE *fp = fopen(path, "r");
    if (!fp)
        return SNG_EIO;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), fp)) > 0)
        text.append(buf, got);
    const bool read_ok = !ferror(fp);
    fclose(fp);
    if (!read_ok)
        return SNG_EIO;
    std::istringstream in(text);
    std::string line;
    if (!std::getline(in, line) || line != kTuneFileHeader)
        return SNG_EINVAL;
    std::map<TuneKey, sng_config> add;
    while (std::getline(in, line)) {
        if (line.empty())
            continue;
        std::istringstream ls(line);
        TuneKey k;
        sng_config c;
        int32_t *f = reinterpret_cast<int32_t *>(&c);
        if (!(ls >> k.form >> k.d >> k.vec >> k.lg_n >> k.lg_m))
            return SNG_EINVAL;
        for (int i = 0; i < kConfigFields; ++i)
            if (!(ls >> f[i]))
                return SNG_EINVAL;
        std::string rest;
        if (ls >> rest)
            return SNG_EINVAL;  // trailing fields
        if (k.form < kFormPlain || k.form > kFormBatch || k.d < 1 || k.vec < 0 || k.vec > 1 ||
            k.lg_n < 0 || k.lg_n > 63 || k.lg_m < 0 || k.lg_m > 63 || check_cfg(&c) != SNG_OK)
            return SNG_EINVAL;
        add[k] = c;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto &kv : add)
        g_tune[kv.first] = kv.second;
    return SNG_OK;
}

}  // extern "C"

namespace {

// sng_cluster with the hook grid given (0: the tuned or default one).
int cluster_run(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                uint64_t seed, int32_t min_pts, const uint32_t *degrees, int32_t *labels,
                void *workspace, size_t ws_bytes, void *stream, unsigned hook_blocks)
{
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if ((rc = check_eps(eps))) return rc;
    if (m < 0) return SNG_EINVAL;
    if (m > kMaxM) return SNG_ERANGE;
    if (n > 0 && (!degrees || !labels)) return SNG_EINVAL;
    const size_t need = plain_ws_bytes(n, m);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, eps, seed, min_pts);
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    (void)cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    I.mask = cv.take<uint32_t>(sizes_for(n, m).chunks * 8);
    I.deg = const_cast<uint32_t *>(degrees);  // read only below
    I.labels = labels;
    if (hook_blocks == 0) {
        sng_config tuned;
        if (tuned_entry(tune_key(X, d, ld, n, m), &tuned))
            hook_blocks = (unsigned)tuned.hook_blocks;
    }
    SNG_TRY(launch_fill_u64(I.cnt + kCntCore, 3, 0ull, st));  // core/cluster/noise counts
    SNG_TRY(launch_core_init(I, st));
    if (I.m > 0)
        SNG_TRY(launch_hook_mask(I, st, hook_blocks));
    SNG_TRY(launch_finalize(I, st));
    return SNG_OK;
}

}  // namespace

extern "C" {

int sng_cluster(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                uint64_t seed, int32_t min_pts, const uint32_t *degrees, int32_t *labels,
                void *workspace, size_t ws_bytes, void *stream)
{
    return cluster_run(X, n, d, ld, m, eps, seed, min_pts, degrees, labels, workspace, ws_bytes,
                       stream, 0u);
}

int sng_autotune_hook(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                      uint64_t seed, int32_t min_pts, const uint32_t *degrees, int32_t *labels,
                      void *workspace, size_t ws_bytes, int32_t trials, sng_config *best,
                      float *best_ms, int32_t *tried, void *stream)
{
    if (!best || trials < 1 || trials > 1000) return SNG_EINVAL;
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    memset(best, 0, sizeof(*best));
    if (best_ms) *best_ms = 0.0f;
    if (tried) *tried = 0;
    // grids around the default's cap of 4096 blocks of 256 threads
    std::vector<sng_config> cand;
    for (int b : {1024, 2048, 4096, 8192, 16384, 32768}) {
        sng_config c;
        memset(&c, 0, sizeof(c));
        c.hook_blocks = b;
        cand.push_back(c);
    }
    rc = tune_candidates(
        cand, (hipStream_t)stream, trials,
        [&](const sng_config &c) {
            return cluster_run(X, n, d, ld, m, eps, seed, min_pts, degrees, labels, workspace,
                               ws_bytes, stream, (unsigned)c.hook_blocks);
        },
        best, best_ms, tried);
    if (rc != SNG_OK)
        return rc;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    sng_config &e = g_tune[tune_key(X, d, ld, n, m)];  // zero-initialised when new
    e.hook_blocks = best->hook_blocks;
    return SNG_OK;
}

int sng_dbscan(const float *X, int64_t n, int32_t d, int64_t ld, double s, double eps,
               int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
               void *workspace, size_t ws_bytes, const sng_config *cfg, void *stream)
{
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if ((rc = check_eps(eps))) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    int64_t m = 0;
    if ((rc = m_from_s(s, n, &m))) return rc;
    if (n > 0 && !labels) return SNG_EINVAL;
    if (n > 0 && (((uintptr_t)labels & 3u) || ((uintptr_t)degrees & 3u))) return SNG_EINVAL;
    if ((rc = check_simple(cfg, n, m))) return rc;
    const size_t need =
        plain_ws_bytes(n, m) + (cfg && cfg->simple_graph ? simple_ws_bytes(n, m) : 0);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, eps, seed, min_pts);
    I.out_deg = (cfg && cfg->out_degree) ? 1 : 0;
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    uint32_t *wdeg = cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    I.mask = cv.take<uint32_t>(sizes_for(n, m).chunks * 8);
    const SimpleTable simple = carve_simple(cv, cfg, n, m);
    I.deg = degrees ? degrees : wdeg;
    I.labels = labels;
    sng_config tuned;
    cfg = effective_cfg(I, cfg, &tuned);
    BucketGeom B;
    bool use = false;
    const uint32_t layout = simple.table ? kLayoutPlain | kLayoutSimpleTable : kLayoutPlain;
    if ((rc = pick_bucket(I, cfg, workspace, ws_bytes, cv.off, &B, &use, layout))) return rc;
    return run_plain(I, cfg, true, use ? &B : nullptr, st, nullptr, simple);
}

int sng_similarity_workspace_size(int64_t n, int32_t d, int64_t m, int32_t kind, int32_t flags,
                                  size_t *bytes)
{
    if (!bytes || n < 0 || d < 1 || m < 0 || (flags & ~(SNG_WS_DIRECT | SNG_WS_SIMPLE_GRAPH)) ||
        (kind != SNG_SIM_DOT && kind != SNG_SIM_COSINE))
        return SNG_EINVAL;
    if (n > kMaxN || m > kMaxM)
        return SNG_ERANGE;
    if ((flags & SNG_WS_SIMPLE_GRAPH) && simple_table_log2(n, m) > kSimpleMaxLog2)
        return SNG_ERANGE;
    size_t b = sim_ws_bytes(n, d, m, kind) +
               ((flags & SNG_WS_SIMPLE_GRAPH) ? simple_ws_bytes(n, m) : 0);
    BucketGeom g;
    if (!(flags & SNG_WS_DIRECT) && bucket_geometry(n, d, m, true, &g))
        b = align_up(b + bucket_bytes(g));
    *bytes = b;
    return SNG_OK;
}

int sng_dbscan_similarity(const float *X, int64_t n, int32_t d, int64_t ld, double s,
                          int32_t kind, double tau, int32_t min_pts, uint64_t seed,
                          int32_t *labels, uint32_t *degrees, void *workspace, size_t ws_bytes,
                          const sng_config *cfg, void *stream)
{
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if (kind != SNG_SIM_DOT && kind != SNG_SIM_COSINE) return SNG_EINVAL;
    if (isnan(tau) || isinf(tau)) return SNG_EINVAL;
    if ((rc = check_cfg(cfg))) return rc;
    if (cfg && cfg->reuse_sample) return SNG_EINVAL;  // the sample is not kept in this layout
    int64_t m = 0;
    if ((rc = m_from_s(s, n, &m))) return rc;
    if (n > 0 && !labels) return SNG_EINVAL;
    if (n > 0 && (((uintptr_t)labels & 3u) || ((uintptr_t)degrees & 3u))) return SNG_EINVAL;
    if ((rc = check_simple(cfg, n, m))) return rc;
    const size_t need =
        sim_ws_bytes(n, d, m, kind) + (cfg && cfg->simple_graph ? simple_ws_bytes(n, m) : 0);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, 0.0, seed, min_pts);
    I.out_deg = (cfg && cfg->out_degree) ? 1 : 0;
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    uint32_t *wdeg = cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    I.mask = cv.take<uint32_t>(sizes_for(n, m).chunks * 8);
    float *rows = cv.take<float>(sim_rows_floats(n, d, kind));
    const SimpleTable simple = carve_simple(cv, cfg, n, m);
    I.deg = degrees ? degrees : wdeg;
    I.labels = labels;
    SimRows sim;
    sim.unit = rows;
    set_similarity(I, kind, tau, sim.unit);
    sng_config tuned;
    cfg = effective_cfg(I, cfg, &tuned);
    BucketGeom B;
    bool use = false;
    const uint32_t layout =
        simple.table ? kLayoutSimilarity | kLayoutSimpleTable : kLayoutSimilarity;
    if ((rc = pick_bucket(I, cfg, workspace, ws_bytes, cv.off, &B, &use, layout))) return rc;
    return run_plain(I, cfg, true, use ? &B : nullptr, st, &sim, simple);
}

int sng_dbscan_lowp(const float *X, int64_t n, int32_t d, int64_t ld, const uint16_t *X_lp,
                    int64_t ld_lp, float lp_scale, int32_t prec, double s, double eps,
                    int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
                    void *workspace, size_t ws_bytes, const sng_config *cfg, void *stream)
{
    if (cfg && cfg->reuse_sample)
        return SNG_EINVAL;  // the mixed form draws its own sample
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if (cfg && cfg->simple_graph) return SNG_ENOTIMPL;
    if ((rc = check_eps(eps))) return rc;
    if (prec != SNG_BF16 && prec != SNG_FP16) return SNG_EINVAL;
    if (!(lp_scale == lp_scale) || __builtin_isinf(lp_scale) || lp_scale == 0.0f) return SNG_EINVAL;
    if (n > 0 && (!X_lp || ((uintptr_t)X_lp & 15u) || ld_lp < d || (ld_lp & 7))) return SNG_EINVAL;
    if (d > 16384) return SNG_ENOTIMPL;
    int64_t m = 0;
    if ((rc = m_from_s(s, n, &m))) return rc;
    if (n > 0 && !labels) return SNG_EINVAL;
    if (n > 0 && (((uintptr_t)labels & 3u) || ((uintptr_t)degrees & 3u))) return SNG_EINVAL;
    const size_t need = lowp_ws_bytes(n, m);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, eps, seed, min_pts);
    I.out_deg = (cfg && cfg->out_degree) ? 1 : 0;
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    uint32_t *wdeg = cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    const uint64_t words = sizes_for(n, m).chunks * 8;
    I.mask = cv.take<uint32_t>(words);
    I.deg = degrees ? degrees : wdeg;
    I.labels = labels;
    LowpArgs L;
    memset(&L, 0, sizeof(L));
    L.Xlp = X_lp;
    L.ld_lp = ld_lp;
    L.scale = lp_scale;
    L.scale2 = (double)lp_scale * (double)lp_scale;
    L.stats = cv.take<double>((size_t)n * 4);
    L.queue = cv.take<uint64_t>((size_t)n * (size_t)m);
    L.qcap = (uint64_t)n * (uint64_t)m;
    // FP32 accumulation of d exact products in any order, each rounding
    // allowed twice the round-to-nearest error (directed rounding included)
    const double ua = 0x1p-22;
    L.gamma_acc = d * ua < 0.5 ? d * ua / (1.0 - d * ua) : 1e300;
    L.gamma_norm = (2.0 * d + 24.0) * 0x1p-52;
    L.tiny = (2.0 * d + 2.0) * 0x1p-126;
    // error of the binary64 definition: |D - S| <= c*S + beta64
    const double c = (d + 3.0) * 0x1p-53 / (1.0 - (d + 3.0) * 0x1p-53);
    const double beta64 = (2.0 * d + 2.0) * 0x1p-1074;
    L.eps2_lo = (I.eps2 - beta64) / (1.0 + c) * (1.0 - 0x1p-50);
    L.eps2_hi = (I.eps2 + beta64) / (1.0 - c) * (1.0 + 0x1p-50);
    SNG_TRY(init_header(I.cnt, (uint64_t)n * (uint64_t)m, c, st));
    sng_config tuned;
    const sng_config *ec =
        effective_cfg(I, cfg, &tuned, prec == SNG_BF16 ? kFormBf16 : kFormFp16);
    SNG_TRY(launch_fill_u32(I.deg, I.n, 0u, st));
    SNG_TRY(launch_fill_u32(I.mask, words, 0u, st));
    const hipError_t le =
        launch_lowp(I, L, prec, st, ec ? ec->mfma_waves : 0, ec ? ec->mfma_ksteps : 0);
    if (le == hipErrorInvalidValue && ec && ec->mfma_waves != 0)
        return SNG_ENOTIMPL;  // the requested waves per block do not fit the LDS for this d
    SNG_TRY(le);
    SNG_TRY(launch_core_init(I, st));
    if (I.m > 0)
        SNG_TRY(launch_hook_mask(I, st, ec ? (unsigned)ec->hook_blocks : 0u));
    SNG_TRY(launch_finalize(I, st));
    return SNG_OK;
}

int sng_autotune_lowp(const float *X, int64_t n, int32_t d, int64_t ld, const uint16_t *X_lp,
                      int64_t ld_lp, float lp_scale, int32_t prec, double s, double eps,
                      int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
                      void *workspace, size_t ws_bytes, int32_t trials, sng_config *best,
                      float *best_ms, int32_t *tried, void *stream)
{
    if (!best || trials < 1 || trials > 1000) return SNG_EINVAL;
    if (prec != SNG_BF16 && prec != SNG_FP16) return SNG_EINVAL;
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    int64_t m = 0;
    if ((rc = m_from_s(s, n, &m))) return rc;
    memset(best, 0, sizeof(*best));
    if (best_ms) *best_ms = 0.0f;
    if (tried) *tried = 0;
    if (n == 0 || m == 0)
        return SNG_OK;  // no sampled-distance pass to tune
    std::vector<sng_config> cand;
    for (int w : {4, 2, 1})
        for (int k : {4, 8, 16}) {
            sng_config c;
            memset(&c, 0, sizeof(c));
            c.mfma_waves = w;
            c.mfma_ksteps = k;
            cand.push_back(c);
        }
    rc = tune_candidates(
        cand, (hipStream_t)stream, trials,
        [&](const sng_config &c) {
            return sng_dbscan_lowp(X, n, d, ld, X_lp, ld_lp, lp_scale, prec, s, eps, min_pts,
                                   seed, labels, degrees, workspace, ws_bytes, &c, stream);
        },
        best, best_ms, tried);
    if (rc != SNG_OK)
        return rc;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[tune_key(X, d, ld, n, m, prec == SNG_BF16 ? kFormBf16 : kFormFp16)] = *best;
    return SNG_OK;
}

int sng_graph_workspace_size(int64_t n, size_t *bytes)
{
    if (!bytes || n < 0)
        return SNG_EINVAL;
    if (n > kMaxN)
        return SNG_ERANGE;
    *bytes = align_up(align_up(kHeaderBytes + (size_t)n * 4) + (size_t)n);
    return SNG_OK;
}

int sng_graph_labels(int64_t n, const int32_t *edges, int64_t n_edges, int32_t min_pts,
                     int32_t *labels, uint32_t *degrees, void *workspace, size_t ws_bytes,
                     void *stream)
{
    if (n < 0 || n_edges < 0 || (n_edges > 0 && !edges) || (n > 0 && !labels))
        return SNG_EINVAL;
    if (n > kMaxN)
        return SNG_ERANGE;
    if (n == 0 && n_edges > 0)
        return SNG_EINVAL;
    size_t need = 0;
    sng_graph_workspace_size(n, &need);
    if (!workspace || ws_bytes < need)
        return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I;
    memset(&I, 0, sizeof(I));
    I.n = (uint32_t)n;
    I.min_pts = min_pts;
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    uint32_t *wdeg = cv.take<uint32_t>((size_t)n);
    I.core = cv.take<uint8_t>((size_t)n);
    I.deg = degrees ? degrees : wdeg;
    I.labels = labels;
    SNG_TRY(init_header(I.cnt, (uint64_t)n_edges, 0.0, st));
    SNG_TRY(launch_fill_u32(I.deg, I.n, 0u, st));
    SNG_TRY(launch_edge_degrees(edges, n_edges, I.deg, st));
    SNG_TRY(launch_core_init(I, st));
    SNG_TRY(launch_hook_edges(I, edges, n_edges, st));
    SNG_TRY(launch_finalize(I, st));
    return SNG_OK;
}

int sng_compact_labels(const int32_t *labels, int64_t n, int32_t *out, int32_t *n_clusters,
                       void *stream)
{
    if (n < 0 || (n > 0 && (!labels || !out)))
        return SNG_EINVAL;
    if (n > kMaxN)
        return SNG_ERANGE;
    if (n > 0) {
        const uintptr_t a0 = (uintptr_t)labels, a1 = a0 + (uintptr_t)n * 4;
        const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (uintptr_t)n * 4;
        if (a0 < b1 && b0 < a1)
            return SNG_EINVAL;  // out must not overlap labels
    }
    SNG_TRY(launch_compact(labels, (uint32_t)n, out, n_clusters, (hipStream_t)stream));
    return SNG_OK;
}

static size_t sweep_ws_bytes(int64_t n, int64_t m, int32_t K, int32_t P)
{
    const Sizes z = sizes_for(n, m);
    size_t b = kHeaderBytes;
    b = align_up(b + (size_t)n * (size_t)K * 4);  // level histograms
    b = align_up(b + z.chunks * 64 * 4);          // level codes per call
    b = align_up(b + (size_t)n * (size_t)P);      // core levels
    b = align_up(b + (size_t)n * (size_t)P * 4);  // level links
    return b;
}

static size_t sweep_ws_bytes_full(int64_t n, int32_t d, int64_t m, int32_t K, int32_t P)
{
    size_t b = sweep_ws_bytes(n, m, K, P);
    BucketGeom g;
    if (bucket_geometry(n, d, m, true, &g))
        b = align_up(b + bucket_bytes(g));
    return b;
}

int sng_sweep_workspace_size(int64_t n, int32_t d, int64_t m, int32_t n_eps, int32_t n_minpts,
                             size_t *bytes)
{
    if (!bytes || n < 0 || d < 1 || m < 0 || n_eps < 1 || n_minpts < 1)
        return SNG_EINVAL;
    if (n > kMaxN || m > kMaxM || n_eps > kSweepMaxK || n_minpts > kSweepMaxP)
        return SNG_ERANGE;
    *bytes = sweep_ws_bytes_full(n, d, m, n_eps, n_minpts);
    return SNG_OK;
}

int sng_dbscan_sweep(const float *X, int64_t n, int32_t d, int64_t ld, double s,
                     const double *eps, int32_t n_eps, const int32_t *min_pts, int32_t n_minpts,
                     uint64_t seed, int32_t *labels, uint32_t *degrees, void *workspace,
                     size_t ws_bytes, const sng_config *cfg, void *stream)
{
    int rc = check_points(X, n, d, ld);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if (cfg && cfg->simple_graph) return SNG_ENOTIMPL;
    if (cfg && cfg->reuse_sample) return SNG_EINVAL;  // its workspace layout differs
    if (!eps || !min_pts || n_eps < 1 || n_minpts < 1) return SNG_EINVAL;
    if (n_eps > kSweepMaxK || n_minpts > kSweepMaxP) return SNG_ERANGE;
    for (int k = 0; k < n_eps; ++k) {
        if ((rc = check_eps(eps[k]))) return rc;
        if (k > 0 && !(eps[k] > eps[k - 1])) return SNG_EINVAL;  // strictly increasing
    }
    int64_t m = 0;
    if ((rc = m_from_s(s, n, &m))) return rc;
    if (n > 0 && !labels) return SNG_EINVAL;
    if ((uint64_t)n * (uint64_t)n_eps * (uint64_t)n_minpts > ((uint64_t)1 << 40)) return SNG_ERANGE;
    const size_t need = sweep_ws_bytes(n, m, n_eps, n_minpts);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    Inst I = make_inst(X, n, d, ld, m, eps[n_eps - 1], seed, 0);
    I.out_deg = (cfg && cfg->out_degree) ? 1 : 0;
    I.cnt = cv.take<unsigned long long>(kHeaderBytes / 8);
    SweepArgs S;
    memset(&S, 0, sizeof(S));
    S.K = n_eps;
    S.P = n_minpts;
    for (int k = 0; k < n_eps; ++k) {
        S.c.e2[k] = eps[k] * eps[k];
        band_fp32(S.c.e2[k], d, &S.c.lo[k], &S.c.hi[k], nullptr);
    }
    for (int p = 0; p < n_minpts; ++p)
        S.c.min_pts[p] = min_pts[p];
    S.hist = cv.take<uint32_t>((size_t)n * n_eps);
    S.codes = cv.take<uint32_t>(sizes_for(n, m).chunks * 64);
    S.kc = cv.take<uint8_t>((size_t)n * n_minpts);
    S.link = cv.take<int32_t>((size_t)n * n_minpts);
    S.labels = labels;
    S.degrees = degrees;
    double band = 0.0;
    {
        float lo, hi;
        band_fp32(S.c.e2[n_eps - 1], d, &lo, &hi, &band);
    }
    BucketGeom B;
    bool use = false;
    sng_config tuned;
    cfg = effective_cfg(I, cfg, &tuned);
    if ((rc = pick_bucket(I, cfg, workspace, ws_bytes, cv.off, &B, &use, kLayoutSweep))) return rc;
    SNG_TRY(init_header(I.cnt, (uint64_t)n * (uint64_t)m, band, st));
    SNG_TRY(launch_fill_u32(S.hist, (uint64_t)n * n_eps, 0u, st));
    SNG_TRY(launch_sweep(I, S, shape_for(I, cfg, use), use ? &B : nullptr, st));
    return SNG_OK;
}

}  // extern "C"

namespace {

// Host-side image of a batch: descriptors, prefix tables and where they go
// in the workspace.
struct BatchHost {
    std::vector<Inst> insts;
    std::vector<uint64_t> chunk_starts, pblk, wblk;
    BatchGeom G;
    Inst *dT = nullptr;
    uint64_t *dChunk = nullptr, *dP = nullptr, *dW = nullptr;
    bool vec_ok = true;
    int d = 0;
};

size_t batch_layout(int32_t count, const int64_t *n, const int64_t *m, size_t *mask_words)
{
    size_t b = align_up((size_t)count * kInstHeader);
    b = align_up(b < kHeaderBytes ? kHeaderBytes : b);
    b = align_up(b + (size_t)count * sizeof(Inst));
    b = align_up(b + 3 * (size_t)(count + 1) * sizeof(uint64_t));
    uint64_t chunks = 0;
    for (int k = 0; k < count; ++k) {
        b = align_up(b + (size_t)n[k] * 4);
        b = align_up(b + (size_t)n[k]);
        chunks += sizes_for(n[k], m[k]).chunks;
    }
    b = align_up(b + chunks * 8 * 4);
    if (mask_words)
        *mask_words = chunks * 8;
    return b;
}

int batch_prepare(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                  const int64_t *ld, const double *s, const double *eps, const int32_t *min_pts,
                  const uint64_t *seed, int32_t *const *labels, uint32_t *const *degrees,
                  void *workspace, size_t ws_bytes, BatchHost &h)
{
    if (count < 0 || (count > 0 && (!X || !n || !ld || !s || !eps || !min_pts || !seed || !labels)))
        return SNG_EINVAL;
    if (count > (1 << 20)) return SNG_ERANGE;
    if (d < 1) return SNG_EINVAL;
    std::vector<int64_t> ms(count);
    for (int k = 0; k < count; ++k) {
        int rc = check_points(X[k], n[k], d, ld[k]);
        if (rc) return rc;
        if ((rc = check_eps(eps[k]))) return rc;
        if ((rc = m_from_s(s[k], n[k], &ms[k]))) return rc;
        if (n[k] > 0 && (!labels[k] || ((uintptr_t)labels[k] & 3u))) return SNG_EINVAL;
        if (degrees && ((uintptr_t)degrees[k] & 3u)) return SNG_EINVAL;
    }
    size_t words = 0;
    const size_t need = batch_layout(count, n, ms.data(), &words);
    if (!workspace || ws_bytes < need) return SNG_EWORKSPACE;
    Carve cv(workspace);
    char *headers = cv.take<char>((size_t)count * kInstHeader < kHeaderBytes
                                      ? kHeaderBytes : (size_t)count * kInstHeader);
    h.dT = cv.take<Inst>((size_t)count);
    h.dChunk = cv.take<uint64_t>(3 * (size_t)(count + 1));
    h.dP = h.dChunk + (count + 1);
    h.dW = h.dP + (count + 1);
    h.insts.resize(count);
    h.chunk_starts.assign(count + 1, 0);
    h.pblk.assign(count + 1, 0);
    h.wblk.assign(count + 1, 0);
    h.d = d;
    uint64_t chunk = 0, pb = 0, wb = 0;
    std::vector<uint32_t *> wdeg(count);
    std::vector<uint8_t *> core(count);
    for (int k = 0; k < count; ++k) {
        wdeg[k] = cv.take<uint32_t>((size_t)n[k]);
        core[k] = cv.take<uint8_t>((size_t)n[k]);
    }
    uint32_t *mask = cv.take<uint32_t>(words);
    for (int k = 0; k < count; ++k) {
        Inst I = make_inst(X[k], n[k], d, ld[k], ms[k], eps[k], seed[k], min_pts[k]);
        I.cnt = reinterpret_cast<unsigned long long *>(headers + (size_t)k * kInstHeader);
        I.deg = (degrees && degrees[k]) ? degrees[k] : wdeg[k];
        I.core = core[k];
        I.mask = mask;
        I.labels = labels[k];
        I.chunk0 = chunk;
        h.chunk_starts[k] = chunk;
        h.pblk[k] = pb;
        h.wblk[k] = wb;
        chunk += I.chunks;
        const uint64_t nblk = ((uint64_t)n[k] + kPointsPerBlock - 1) / kPointsPerBlock;
        pb += nblk ? nblk : 1;
        wb += (I.chunks * 8 + kWordsPerBlock - 1) / kWordsPerBlock;
        if (((uintptr_t)X[k] % 16) || (ld[k] % 4))
            h.vec_ok = false;
        h.insts[k] = I;
    }
    h.chunk_starts[count] = chunk;
    h.pblk[count] = pb;
    h.wblk[count] = wb;
    h.G.count = count;
    h.G.pblk = h.dP;
    h.G.wblk = h.dW;
    h.G.chunk_starts = h.dChunk;
    h.G.total_pblocks = pb;
    h.G.total_wblocks = wb;
    h.G.total_chunks = chunk;
    if (pb > 0x7FFFFFFFull || wb > 0x7FFFFFFFull) return SNG_ERANGE;
    return SNG_OK;
}

// Host tables -> workspace. `sync` true: blocking copies (plan creation);
// false: copies on `st`, then waits for them so the host tables may go.
int batch_upload(const BatchHost &h, hipStream_t st)
{
    const int count = h.G.count;
    if (count == 0)
        return SNG_OK;
    if (hipMemcpyAsync(h.dT, h.insts.data(), count * sizeof(Inst), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(h.dChunk, h.chunk_starts.data(), (count + 1) * sizeof(uint64_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h.dP, h.pblk.data(), (count + 1) * sizeof(uint64_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h.dW, h.wblk.data(), (count + 1) * sizeof(uint64_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SNG_EHIP;
    return SNG_OK;
}

// A batch's autotune key: d, the row alignment of every instance, and
// ceil(log2) of its largest n and m.
TuneKey batch_key(const BatchHost &h)
{
    uint64_t mn = 0, mm = 0;
    for (const Inst &I : h.insts) {
        mn = I.n > mn ? I.n : mn;
        mm = I.m > mm ? I.m : mm;
    }
    return TuneKey{kFormBatch, h.d, h.vec_ok ? 1 : 0, ceil_log2(mn), ceil_log2(mm)};
}

// The batched pass's launch shape: cfg's, else the tuned one, else the
// defaults.
PassAShape batch_shape(const BatchHost &h, const sng_config *cfg)
{
    sng_config t;
    if (!cfg && tuned_entry(batch_key(h), &t))
        cfg = &t;
    return resolve_shape(h.d, h.vec_ok, cfg ? cfg->lanes_per_pair : 0,
                         cfg ? cfg->chunks_per_wave : 0, 0, cfg ? cfg->prefetch : 0);
}

}  // namespace

struct sng_batch_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;
};

extern "C" {

int sng_batch_workspace_size(int32_t count, const int64_t *n, int32_t d, const double *s,
                             size_t *bytes)
{
    if (!bytes || count < 0 || (count > 0 && (!n || !s)) || d < 1)
        return SNG_EINVAL;
    std::vector<int64_t> ms(count);
    for (int k = 0; k < count; ++k) {
        if (n[k] < 0) return SNG_EINVAL;
        if (n[k] > kMaxN) return SNG_ERANGE;
        const int rc = m_from_s(s[k], n[k], &ms[k]);
        if (rc) return rc;
    }
    *bytes = batch_layout(count, n, ms.data(), nullptr);
    return SNG_OK;
}

int sng_dbscan_batch(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                     const int64_t *ld, const double *s, const double *eps,
                     const int32_t *min_pts, const uint64_t *seed, int32_t *const *labels,
                     uint32_t *const *degrees, void *workspace, size_t ws_bytes, void *stream)
{
    BatchHost h;
    int rc = batch_prepare(count, X, n, d, ld, s, eps, min_pts, seed, labels, degrees, workspace,
                           ws_bytes, h);
    if (rc) return rc;
    if (count == 0) return SNG_OK;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = batch_upload(h, st))) return rc;
    const PassAShape sh = batch_shape(h, nullptr);
    SNG_TRY(launch_batch(h.dT, h.G, d, h.vec_ok, sh, st));
    return SNG_OK;
}

int sng_autotune_batch(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                       const int64_t *ld, const double *s, const double *eps,
                       const int32_t *min_pts, const uint64_t *seed, int32_t *const *labels,
                       uint32_t *const *degrees, void *workspace, size_t ws_bytes, int32_t trials,
                       sng_config *best, float *best_ms, int32_t *tried, void *stream)
{
    if (!best || trials < 1 || trials > 1000) return SNG_EINVAL;
    BatchHost h;
    int rc = batch_prepare(count, X, n, d, ld, s, eps, min_pts, seed, labels, degrees, workspace,
                           ws_bytes, h);
    if (rc) return rc;
    memset(best, 0, sizeof(*best));
    if (best_ms) *best_ms = 0.0f;
    if (tried) *tried = 0;
    if (count == 0) return SNG_OK;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = batch_upload(h, st))) return rc;
    // lanes per pair around the default, rows in flight, chunks per wave;
    // shapes that resolve to the same launch are tried once
    const int g0 = resolve_shape(d, h.vec_ok, 0, 0, 0, 0).lanes;
    std::vector<sng_config> cand;
    std::vector<std::tuple<int, int, int>> seen;
    for (int g : {g0, g0 / 2, g0 * 2}) {
        if (g < 1 || g > 64) continue;
        for (int pf : {4, 8, 16})
            for (int cpw : {4, 8, 16, 32}) {
                const PassAShape sh = resolve_shape(d, h.vec_ok, g, cpw, 0, pf);
                const auto key = std::make_tuple(sh.lanes, sh.chunks_per_wave, sh.owners_per_batch);
                bool dup = false;
                for (const auto &k : seen)
                    dup = dup || k == key;
                if (dup) continue;
                seen.push_back(key);
                sng_config c;
                memset(&c, 0, sizeof(c));
                c.lanes_per_pair = sh.lanes;
                c.chunks_per_wave = sh.chunks_per_wave;
                c.prefetch = 4 * sh.owners_per_batch;
                cand.push_back(c);
            }
    }
    rc = tune_candidates(
        cand, st, trials,
        [&](const sng_config &c) {
            return hip_rc(launch_batch(h.dT, h.G, d, h.vec_ok, batch_shape(h, &c), st));
        },
        best, best_ms, tried);
    if (rc != SNG_OK)
        return rc;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[batch_key(h)] = *best;
    return SNG_OK;
}

int sng_batch_plan_create(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                          const int64_t *ld, const double *s, const double *eps,
                          const int32_t *min_pts, const uint64_t *seed, int32_t *const *labels,
                          uint32_t *const *degrees, void *workspace, size_t ws_bytes,
                          void *stream, sng_batch_plan **plan)
{
    if (!plan) return SNG_EINVAL;
    *plan = nullptr;
    BatchHost h;
    int rc = batch_prepare(count, X, n, d, ld, s, eps, min_pts, seed, labels, degrees, workspace,
                           ws_bytes, h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = batch_upload(h, st))) return rc;
    sng_batch_plan *p = new sng_batch_plan();
    if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return SNG_EHIP;
    }
    const PassAShape sh = batch_shape(h, nullptr);
    bool ok = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
    hipError_t le = hipSuccess;
    if (ok)
        le = launch_batch(h.dT, h.G, d, h.vec_ok, sh, p->capture);
    if (ok)
        ok = hipStreamEndCapture(p->capture, &p->graph) == hipSuccess && le == hipSuccess;
    if (ok)
        ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        sng_batch_plan_destroy(p);
        return SNG_EHIP;
    }
    *plan = p;
    return SNG_OK;
}

int sng_batch_plan_launch(sng_batch_plan *plan, void *stream)
{
    if (!plan || !plan->exec)
        return SNG_EINVAL;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? SNG_OK : SNG_EHIP;
}

int sng_batch_plan_destroy(sng_batch_plan *plan)
{
    if (!plan)
        return SNG_OK;
    // Teardown is best effort: each handle is released even if another fails.
    hipError_t e = hipSuccess, x;
    if (plan->exec && (x = hipGraphExecDestroy(plan->exec)) != hipSuccess)
        e = x;
    if (plan->graph && (x = hipGraphDestroy(plan->graph)) != hipSuccess)
        e = x;
    if (plan->capture && (x = hipStreamDestroy(plan->capture)) != hipSuccess)
        e = x;
    delete plan;
    return e == hipSuccess ? SNG_OK : SNG_EHIP;
}

int sng_stats_read(const void *workspace, int32_t index, sng_stats *out, void *stream)
{
    if (!workspace || !out || index < 0)
        return SNG_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess)
        return SNG_EHIP;
    unsigned long long h[kFltEnd];
    const char *src = (const char *)workspace + (size_t)index * kInstHeader;
    if (hipMemcpy(h, src, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return SNG_EHIP;
    out->slots = h[kCntSlots];
    out->self_pairs = h[kCntSelf];
    out->accepted = h[kCntAccepted];
    out->rechecked = h[kCntRechecked];
    out->n_core = h[kCntCore];
    out->n_clusters = h[kCntClusters];
    out->n_noise = h[kCntNoise];
    out->overflow = h[kCntOverflow];
    memcpy(&out->band_rel, &h[kCntNum], sizeof(double));
    out->filter_gamma = out->filter_r_max = out->filter_r_mean = out->filter_rel_width = 0.0;
    double f[kFltEnd - kFltGamma];
    memcpy(f, &h[kFltGamma], sizeof(f));
    const uint64_t rows = h[kFltRows];
    if (f[0] > 0.0 && rows > 0) {  // a mixed-form call: derive its filter's width
        const double gamma = f[0], gamma_norm = f[kFltGammaNorm - kFltGamma];
        const double scale2 = f[kFltScale2 - kFltGamma], eps2 = f[kFltEps2 - kFltGamma];
        const double r_mean = f[kFltRSum - kFltGamma] / (double)rows;
        const double a_mean = f[kFltASum - kFltGamma] / (double)rows;
        out->filter_gamma = gamma;
        out->filter_r_max = f[kFltRMax - kFltGamma];
        out->filter_r_mean = r_mean;
        // two rows of norm a and radius r at distance eps: the copy's squared
        // distance is known within scale^2 * 2a^2 (gamma + gamma_norm), i.e. its
        // distance within half that over eps, and the rows within 2r of the copies
        const double eps = sqrt(eps2);
        out->filter_rel_width =
            eps > 0.0 ? (2.0 * r_mean + scale2 * a_mean * a_mean * (gamma + gamma_norm) / eps) / eps
                      : HUGE_VAL;
        out->band_rel = out->filter_rel_width;
    }
    return out->overflow ? SNG_EOVERFLOW : SNG_OK;
}

}  // extern "C"
