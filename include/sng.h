/*
 * sng.h -- C ABI of the MI355X (gfx950) SNG-DBSCAN library, libsng.so.
 *
 * SNG-DBSCAN (Jiang, Jang, Lacki, "Faster DBSCAN via subsampled similarity
 * queries", NeurIPS 2020) clusters points X[n,d] from a subsampled
 * eps-neighbourhood graph (Algorithm 1, Section 3): every point queries
 * ceil(s*n) sampled partners, a pair closer than eps becomes an edge, points of
 * degree >= MinPts are core points, the connected components of the core
 * points are the clusters, a non-core point joins a cluster it touches, and
 * the rest is noise.
 *
 * What this library computes, exactly (the readings that make the output
 * unique; Algorithm 1 leaves these open):
 *   m        = ceil(fl64(s * n)) samples per point (calls that take m
 *            directly accept any 0 <= m <= 2^31).
 *   sample t of point i (t < m) is j = W[t mod 4] mod n, where
 *            W = Philox4x32-10(counter = (t/4, i, 0, 0),
 *                              key = (seed mod 2^32, seed / 2^32))
 *            (Salmon, Moraes, Dror, Shaw, SC'11).
 *   edge     (i, j) iff j != i and D(i,j) <= fl64(eps*eps), with D the squared
 *            Euclidean distance evaluated in binary64: acc = 0; for k < d in
 *            order: delta = (double)x_ik - (double)x_jk; acc += delta*delta,
 *            every operation rounded to nearest-even, no fused multiply-add.
 *            NaN never forms an edge. (sng_dbscan_similarity: a dot-product
 *            or cosine threshold instead, defined there.)
 *   degree   symmetrised multigraph degree: each accepted sample adds one to
 *            both endpoints (a pair sampled twice counts twice); the
 *            out_degree and simple_graph fields of sng_config select the
 *            out-degree or the number of distinct neighbours instead.
 *   core     (int64)degree >= MinPts (MinPts <= 0 makes every point core).
 *   label    core point: smallest index of its core component;
 *            non-core point: label of its smallest-index core neighbour;
 *            otherwise -1 (noise).
 * Results are bit-exact and deterministic for every stream, launch shape and
 * tuning choice; the reduced-precision path returns the same labels.
 *
 * Conventions for every call:
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory. The caller owns all buffers.
 *   - X is row-major: element (i,k) at X[i*ld + k], ld >= d, 4-byte aligned,
 *     and readable for n*ld floats (rows may be read in 16-byte pieces up to
 *     the next multiple of four floats when ld is a multiple of four).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls enqueue work on it and return without waiting; outputs are valid
 *     once the stream has been synchronised. sng_dbscan and
 *     sng_dbscan_similarity enqueue kernels only (no memset, allocation or
 *     host wait), so a call may be recorded into a HIP graph and replayed;
 *     each replay recomputes every output from the inputs.
 *   - Arguments are validated before anything is enqueued; a call that
 *     returns a validation error has written nothing. SNG_EHIP reports a HIP
 *     call or launch that failed after earlier work was enqueued.
 *   - `workspace` is device memory of at least the size reported by the
 *     matching *_workspace_size call; its contents on entry are ignored,
 *     except where a call is asked to continue from an earlier one
 *     (sng_cluster, reuse_sample). One workspace must not be used by two
 *     calls in flight at once.
 *   - Degrees are 32-bit and wrap beyond 2^32-1 (unreachable in practice:
 *     the expected degree is about 2m).
 */
#ifndef SNG_H
#define SNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SNG_OK = 0,
    SNG_EINVAL = -1,     /* invalid argument (null pointer, d < 1, ld < d, eps < 0, ...) */
    SNG_ERANGE = -2,     /* a size beyond what the kernels index (n > 2^31-1, m > 2^31, sweep
                            grids beyond 64 eps or 16 MinPts values, ...) */
    SNG_EWORKSPACE = -3, /* workspace missing or smaller than required */
    SNG_EHIP = -4,       /* a HIP runtime call or kernel launch failed */
    SNG_EOVERFLOW = -5,  /* reported by sng_stats_read: a device queue overflowed */
    SNG_ENOTIMPL = -6,   /* requested form not available for these arguments */
    SNG_EIO = -7         /* a file could not be opened, read or written */
} sng_status;

typedef enum {
    SNG_FP32 = 0, /* plain form: binary32 filter, binary64 recheck near eps */
    SNG_BF16 = 1, /* mixed form: bfloat16 copy on MFMA, binary64 recheck */
    SNG_FP16 = 2  /* mixed form: float16 copy on MFMA, binary64 recheck */
} sng_precision;

/* Launch shape of the sampled-distance pass. Zero fields mean "library
 * default"; every choice gives identical results. */
typedef struct {
    int32_t lanes_per_pair;  /* 1,2,4,8,16,32,64 lanes cooperate on one pair */
    int32_t chunks_per_wave; /* 64-call chunks processed by one wavefront */
    int32_t stage_lds;       /* 1: keep the source row in LDS instead of VGPRs */
    int32_t prefetch;        /* partner rows a group gathers ahead: 4, 8 or 16 */
    int32_t schedule;        /* 0 auto, 1 direct gathers, 2 partner-block (L2 reuse) */
    int32_t reuse_sample;    /* 1: evaluate the sample sng_sample left in the workspace */
    int32_t out_degree;      /* 1: degree = a point's own accepted samples (see below) */
    int32_t simple_graph;    /* 1: degree = distinct accepted neighbours (see below) */
    int32_t mfma_waves;      /* mixed form: wavefronts per block of the MFMA pass: 1, 2, 4 */
    int32_t mfma_ksteps;     /* mixed form: 32-wide K-steps loaded together: 4, 8, 16 */
    int32_t hook_blocks;     /* post-processing: blocks of the hook launch, 256..65536 */
} sng_config;
/* schedule: the partner-block form sorts the sample slots by partner block
 * before gathering, so that a block's rows are read from LDS (rows of d <= 8
 * floats: a block is the largest power of two of rows that fits 128 KB, when
 * that gives at most 1024 blocks) or reused from L2 (otherwise: at most 2^16
 * rows fitting 512 KB). It covers d <= 32 and at most 1024 partner blocks
 * (so n <= 2^25 at d = 3, n <= 2^23 at d = 16); auto picks it when it
 * covers the shape, X (n*d*4 bytes) exceeds 8 MB and the workspace holds its
 * records, direct gathers otherwise. stage_lds implies direct gathers.
 * reuse_sample (sng_degrees and sng_dbscan only; SNG_EINVAL elsewhere and
 * with schedule 1 or stage_lds): skip drawing the partners and evaluate the
 * partner-block sample already in the workspace, as left by sng_sample or by
 * an earlier partner-block call with the same n, d, m and seed (any X of
 * that shape, any eps). The kernels check a tag stored with the sample (it
 * names n, m, seed, block size and workspace layout; calls with other
 * layouts clear it); a missing or different sample does no work and makes
 * sng_stats_read report SNG_EOVERFLOW, and every decoded index is range
 * checked as well. */

/* out_degree (sng_degrees, sng_dbscan, sng_dbscan_lowp, sng_dbscan_sweep):
 * the degree of a point, and so its core test, counts only its own accepted
 * samples (the neighbour count analysed in Lemma 2 of Section 4.1) instead
 * of the symmetrised count; the graph, and so components and borders, is
 * unchanged. The other fields choose a launch shape and never change a
 * result. A config whose launch-shape fields are all zero still runs with
 * the tuned shape of sng_autotune. */

/* simple_graph (sng_degrees, sng_dbscan, sng_dbscan_similarity; SNG_EINVAL
 * together with out_degree or reuse_sample, SNG_ENOTIMPL in the mixed form
 * and the sweep): the sampled graph is read as a simple graph, so the degree
 * of a point, and so its core test, counts its distinct accepted neighbours;
 * a pair sampled several times, by either endpoint, counts once. Components
 * and borders are unchanged. The accepted pairs go through a hash table in
 * the workspace, sized for every slot accepted: 8 * 2^ceil(log2(max(64,
 * 2*n*m))) more bytes (sng_workspace_size with SNG_WS_SIMPLE_GRAPH), and
 * SNG_ERANGE when that exceeds 2^36 entries. Only the part the accepted
 * pairs need is cleared and used. Stats still count accepted slots. */

/* Flags for sng_workspace_size: size for the direct schedule only (smaller;
 * a workspace of that size makes the automatic schedule choose it), and add
 * the table of the simple_graph mode. */
#define SNG_WS_DIRECT 0x100
#define SNG_WS_SIMPLE_GRAPH 0x200

/* Device-side counters, copied out by sng_stats_read. */
typedef struct {
    uint64_t slots;      /* n*m sample slots */
    uint64_t self_pairs; /* slots whose partner is the point itself */
    uint64_t accepted;   /* accepted slots (edges counted with multiplicity) */
    uint64_t rechecked;  /* slots decided by the binary64 recheck */
    uint64_t n_core;
    uint64_t n_clusters;
    uint64_t n_noise;
    uint64_t overflow;   /* non-zero: results invalid (a recheck queue overflowed, or a
                            reused partner-block sample was missing or damaged) */
    double band_rel;     /* relative half-width of the recheck band used: the binary32
                            band around fl64(eps*eps) for the plain form; filter_rel_width
                            for the mixed form (sng_dbscan_lowp) */
    /* The mixed form's filter (sng_dbscan_lowp; zero after other calls). A pair is
     * decided without the binary64 recheck only if eps lies outside
     *   [T_lo - (r_i + r_j), T_hi + (r_i + r_j)],
     * where [T_lo, T_hi] bounds the distance of the 16-bit copies given the binary32
     * MFMA dot product (relative error filter_gamma on the products' magnitudes, plus
     * the binary64 row statistics) and r_i = ||x_i - lp_scale * v_i|| is row i's
     * rounding radius. */
    double filter_gamma;     /* error bound of the binary32 accumulation: d*u/(1-d*u), u = 2^-22 */
    double filter_r_max;     /* largest rounding radius r_i (rounded up) */
    double filter_r_mean;    /* mean rounding radius */
    double filter_rel_width; /* half-width of that interval relative to eps, for two rows of
                                mean norm and mean radius at distance eps */
} sng_stats;

/* Human-readable name of a status code. Never NULL. */
const char *sng_status_string(int status);

/* m = ceil(fl64(s*n)) (Algorithm 1, sampling step). s must be finite and
 * >= 0, n >= 0. Host call, no device work. */
int sng_samples_per_point(double s, int64_t n, int64_t *m);

/* Bytes of workspace for sng_dbscan / sng_degrees / sng_cluster / sng_sample /
 * sng_autotune with n points
 * of dimension d and m samples per point, at precision `prec` (optionally
 * or-ed with SNG_WS_DIRECT). The partner-block schedule keeps 4 bytes per
 * sample slot of records in the workspace. Host call. */
int sng_workspace_size(int64_t n, int32_t d, int64_t m, int32_t prec, size_t *bytes);

/* Sampling step only (Algorithm 1, graph construction; edges are not stored):
 * degrees[n] (device, u32) receives the symmetrised degree of every point.
 * X: device float32 [n, ld]. cfg may be NULL (the tuned configuration of
 * this shape if sng_autotune stored one, else the library's defaults). */
int sng_degrees(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                uint64_t seed, uint32_t *degrees, void *workspace, size_t ws_bytes,
                const sng_config *cfg, void *stream);

/* Sampling step alone (Algorithm 1: each point draws its partners): draws
 * the partner of every sample slot with the partner-block schedule and keeps
 * the slots, sorted by partner block, in the workspace (sized by
 * sng_workspace_size for these n, d, m without SNG_WS_DIRECT). Needs no
 * X: the sample depends on n, d (the block size), m and seed only. Evaluate
 * it with sng_degrees or sng_dbscan and cfg->reuse_sample = 1, as often as
 * wanted. SNG_ENOTIMPL where the partner-block schedule does not apply
 * (d > 32, too many partner blocks). n = 0 or m = 0 is a no-op. */
int sng_sample(int64_t n, int32_t d, int64_t m, uint64_t seed, void *workspace, size_t ws_bytes,
               void *stream);

/* Autotuner of the sampled-distance pass. Runs sng_degrees on the caller's
 * data once per candidate configuration (lanes per pair around the default,
 * 4/8/16 rows in flight, 8 or 16 chunks per wave, LDS staging for wide rows,
 * direct gathers and, where it applies and the workspace holds its records,
 * the partner-block schedule), `trials` timed runs each after one warm-up,
 * timed with HIP events on `stream`, and writes the fastest to *best (host)
 * and its mean time in ms to *best_ms (host, may be NULL); *tried (host, may
 * be NULL) gets the number of candidates timed. Every candidate computes
 * the same degrees. The result is also stored in a process-wide cache
 * (mutex-protected) under the key (d, 16-byte row alignment, ceil(log2 n),
 * ceil(log2 m)); sng_degrees, sng_dbscan and sng_dbscan_sweep calls with
 * cfg == NULL or an all-zero config of that key then run with it (a tuned
 * partner-block schedule falls back to direct gathers when the workspace
 * lacks room). Synchronises the stream. Workspace as for sng_degrees; the
 * degrees it computes stay inside it. n = 0 or m = 0: nothing to tune,
 * *best is all zero. */
int sng_autotune(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                 uint64_t seed, void *workspace, size_t ws_bytes, int32_t trials,
                 sng_config *best, float *best_ms, int32_t *tried, void *stream);
/* The cached configuration for this shape class (X only for its alignment),
 * or SNG_ENOTIMPL when none is cached. Host call. */
int sng_autotune_lookup(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                        sng_config *out);
/* Empties the autotune cache. Host call. */
int sng_autotune_clear(void);

/* The other tuned launch shapes, each timed like sng_autotune (`trials` timed
 * calls per candidate after one warm-up, HIP events on `stream`, which is
 * synchronised; *best, *best_ms, *tried as there) and stored in the same
 * cache under a key that also names the form, so a tuned shape is only used
 * by calls of its own form and precision:
 *   sng_autotune_lowp: sng_dbscan_lowp's arguments; candidates mfma_waves x
 *     mfma_ksteps (the wavefronts per block of the MFMA pass, and how many
 *     32-wide K-steps of partner fragments it loads together). Key (prec, d,
 *     16-byte row alignment, ceil(log2 n), ceil(log2 m)); sng_dbscan_lowp
 *     calls without launch fields of their own then use it.
 *   sng_autotune_hook: sng_cluster's arguments (a sng_degrees call must have
 *     left its accept bits in the workspace); candidates hook_blocks, the
 *     grid of the hook launch. Stored into the plain form's entry of the
 *     shape class (created with default pass fields if there is none), used
 *     by sng_dbscan and sng_cluster.
 *   sng_autotune_batch: sng_dbscan_batch's arguments; candidates lanes per
 *     pair x rows in flight x chunks per wave of the batched pass. Key (d,
 *     row alignment of every instance, ceil(log2 max n), ceil(log2 max m));
 *     sng_dbscan_batch and sng_batch_plan_create then use it.
 * Every candidate computes the same results; labels and degrees hold the
 * last candidate's. */
int sng_autotune_lowp(const float *X, int64_t n, int32_t d, int64_t ld, const uint16_t *X_lp,
                      int64_t ld_lp, float lp_scale, int32_t prec, double s, double eps,
                      int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
                      void *workspace, size_t ws_bytes, int32_t trials, sng_config *best,
                      float *best_ms, int32_t *tried, void *stream);
int sng_autotune_hook(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                      uint64_t seed, int32_t min_pts, const uint32_t *degrees, int32_t *labels,
                      void *workspace, size_t ws_bytes, int32_t trials, sng_config *best,
                      float *best_ms, int32_t *tried, void *stream);
int sng_autotune_batch(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                       const int64_t *ld, const double *s, const double *eps,
                       const int32_t *min_pts, const uint64_t *seed, int32_t *const *labels,
                       uint32_t *const *degrees, void *workspace, size_t ws_bytes, int32_t trials,
                       sng_config *best, float *best_ms, int32_t *tried, void *stream);

/* The autotune cache on disk: sng_autotune_save writes every entry to the
 * text file `path` (replacing it; a header line, then one line per entry:
 * form (0 plain, 1 bfloat16, 2 float16, 3 batch), d, row alignment flag,
 * ceil(log2 n), ceil(log2 m) and the eleven sng_config fields);
 * sng_autotune_load merges such a file into the cache (its entries replace
 * equal keys). A file that does not parse, or holds an invalid
 * configuration, changes nothing and returns SNG_EINVAL; a file that cannot
 * be opened or written returns SNG_EIO. Host calls. */
int sng_autotune_save(const char *path);
int sng_autotune_load(const char *path);

/* Post-processing (Algorithm 1: core points, components of the core
 * subgraph, border assignment) continuing from the accept bits that the last
 * sng_degrees call left in the same workspace (same X, n, d, ld, m, eps and
 * seed must be passed again). degrees: device u32 [n] as filled by that call.
 * Several MinPts values may be clustered from one sng_degrees call. */
int sng_cluster(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m, double eps,
                uint64_t seed, int32_t min_pts, const uint32_t *degrees, int32_t *labels,
                void *workspace, size_t ws_bytes, void *stream);

/* Whole method (Algorithm 1): labels[n] (device, i32) receive the cluster
 * labels; degrees (device, u32 [n]) may be NULL. m = ceil(fl64(s*n)). */
int sng_dbscan(const float *X, int64_t n, int32_t d, int64_t ld, double s, double eps,
               int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
               void *workspace, size_t ws_bytes, const sng_config *cfg, void *stream);

/* Mixed-precision form of sng_dbscan: the sampled dot products run on MFMA
 * from a 16-bit copy X_lp [n, ld_lp] (device, bfloat16 or float16 bit
 * patterns per `prec`) with X ~= lp_scale * X_lp; every pair whose distance is
 * not provably on one side of eps is re-decided in binary64 from X, so
 * labels and degrees equal those of sng_dbscan. X_lp rows must be 16-byte
 * aligned (ld_lp % 8 == 0). */
int sng_dbscan_lowp(const float *X, int64_t n, int32_t d, int64_t ld, const uint16_t *X_lp,
                    int64_t ld_lp, float lp_scale, int32_t prec, double s, double eps,
                    int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
                    void *workspace, size_t ws_bytes, const sng_config *cfg, void *stream);

/* Similarity-threshold form of sng_dbscan. The method needs only a yes/no
 * similarity query per sampled pair (Section 1), so the edge test of the
 * sampling step may be a similarity at least tau instead of a distance at
 * most eps:
 *   SNG_SIM_DOT     <x_i, x_j> >= tau, the binary64 dot product summed in
 *                   coordinate order without fused multiply-adds;
 *   SNG_SIM_COSINE  <x_i, x_j> / (sqrt(<x_i,x_i>) * sqrt(<x_j,x_j>)) >= tau,
 *                   each part as for SNG_SIM_DOT, IEEE square roots, product
 *                   and quotient; a zero row has no cosine and no edge.
 * Sampling, degrees, core points, components and borders are those of
 * sng_dbscan. tau: any finite value (SNG_EINVAL otherwise); kind: one of the
 * two above (SNG_EINVAL otherwise). The binary32 pass filters: the cosine
 * with the squared distance of a unit-length copy of the rows (kept in the
 * workspace), where cos >= tau is |u - v|^2 <= 2 - 2 tau (a row whose
 * squared norm lies outside [2^-100, 2^100] has NaN in the copy); the dot
 * product with the binary32 dot product and the sum of absolute products,
 * which bounds its rounding error. Pairs within the filter's error bound of
 * the threshold, NaN and overflow included, are decided by the binary64
 * definition on the caller's rows, so results equal the definition exactly.
 * Workspace: sng_similarity_workspace_size for the same kind (flags
 * SNG_WS_DIRECT, SNG_WS_SIMPLE_GRAPH as for sng_workspace_size; the cosine
 * adds 4 * n * (d rounded up to a multiple of 4) bytes, the dot product
 * nothing).
 * cfg: launch shape, schedule, out_degree and simple_graph as for
 * sng_dbscan; reuse_sample is not available (SNG_EINVAL). Stats: band_rel is the filter's half-width
 * (cosine: absolute on |u - v|^2; dot product: relative to the sum of
 * absolute products). */
typedef enum {
    SNG_SIM_DOT = 1,
    SNG_SIM_COSINE = 2
} sng_similarity;
int sng_similarity_workspace_size(int64_t n, int32_t d, int64_t m, int32_t kind, int32_t flags,
                                  size_t *bytes);
int sng_dbscan_similarity(const float *X, int64_t n, int32_t d, int64_t ld, double s,
                          int32_t kind, double tau, int32_t min_pts, uint64_t seed,
                          int32_t *labels, uint32_t *degrees, void *workspace, size_t ws_bytes,
                          const sng_config *cfg, void *stream);

/* Compact cluster ids. The method defines its clusters up to a renaming
 * (Section 4.1, Theorem 1); the clustering calls name each cluster by its
 * root, the smallest core index in it. out[i] = the rank of labels[i] among
 * the distinct roots in increasing order (clusters 0..k-1), -1 for noise.
 * labels: device i32 [n] as written by a clustering call (each entry -1 or
 * the index r of a root, labels[r] == r); any other entry maps to -1.
 * out: device i32 [n], must not overlap labels (SNG_EINVAL otherwise).
 * n_clusters: device i32, may be NULL; receives k. No workspace: out holds
 * the intermediate tile counts. */
int sng_compact_labels(const int32_t *labels, int64_t n, int32_t *out, int32_t *n_clusters,
                       void *stream);

/* Post-processing only (Algorithm 1, core points, components and borders) on
 * an explicit list of accepted pairs: edges (device, int32 [n_edges][2]),
 * each pair counted once per occurrence; self-pairs are not allowed.
 * labels[n] and optional degrees[n] are device outputs. */
int sng_graph_workspace_size(int64_t n, size_t *bytes);
int sng_graph_labels(int64_t n, const int32_t *edges, int64_t n_edges, int32_t min_pts,
                     int32_t *labels, uint32_t *degrees, void *workspace, size_t ws_bytes,
                     void *stream);

/* Hyperparameter sweep: every (eps[k], min_pts[p]) pair of a grid from one
 * sampled-distance pass (same sampler for all pairs; Section 5 tunes eps over
 * a grid). eps: host, n_eps values, finite, >= 0 and strictly increasing,
 * 1 <= n_eps <= 64. min_pts: host, 1 <= n_minpts <= 16 values, any int32.
 * More values than these limits: SNG_ERANGE, as when n * n_eps * n_minpts
 * exceeds 2^40. labels: device i32 [n_minpts][n_eps][n]; degrees: device
 * u32 [n_eps][n] or NULL. Each labels[p][k] equals sng_dbscan(..., eps[k],
 * min_pts[p], ...), and degrees[k] its degrees. */
int sng_sweep_workspace_size(int64_t n, int32_t d, int64_t m, int32_t n_eps, int32_t n_minpts,
                             size_t *bytes);
int sng_dbscan_sweep(const float *X, int64_t n, int32_t d, int64_t ld, double s,
                     const double *eps, int32_t n_eps, const int32_t *min_pts, int32_t n_minpts,
                     uint64_t seed, int32_t *labels, uint32_t *degrees, void *workspace,
                     size_t ws_bytes, const sng_config *cfg, void *stream);

/* Batch of independent instances solved together (each equal to its own
 * sng_dbscan call). Arrays of length `count` are host arrays; X[k],
 * labels[k], degrees[k] are device pointers (degrees may be NULL or hold
 * NULL entries). All instances share d; count <= 2^20.
 * Unlike the other calls, sng_dbscan_batch and sng_batch_plan_create copy
 * the batch's instance tables from host memory into the workspace and wait
 * for `stream` to finish that copy (work enqueued on it before the call
 * included) before returning, so neither may be called while `stream` is
 * being captured into a HIP graph; the plan is the captured form. The
 * kernels are enqueued without waiting. */
int sng_batch_workspace_size(int32_t count, const int64_t *n, int32_t d, const double *s,
                             size_t *bytes);
int sng_dbscan_batch(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                     const int64_t *ld, const double *s, const double *eps,
                     const int32_t *min_pts, const uint64_t *seed, int32_t *const *labels,
                     uint32_t *const *degrees, void *workspace, size_t ws_bytes,
                     void *stream);

/* Captured form of sng_dbscan_batch: the plan records every pass of the
 * batch into one HIP graph once; each launch replays it on `stream` with the
 * same buffers (their contents may change between launches) and returns
 * without waiting. */
typedef struct sng_batch_plan sng_batch_plan;
int sng_batch_plan_create(int32_t count, const float *const *X, const int64_t *n, int32_t d,
                          const int64_t *ld, const double *s, const double *eps,
                          const int32_t *min_pts, const uint64_t *seed, int32_t *const *labels,
                          uint32_t *const *degrees, void *workspace, size_t ws_bytes,
                          void *stream, sng_batch_plan **plan);
int sng_batch_plan_launch(sng_batch_plan *plan, void *stream);
/* Releases the plan (always freed; NULL is a no-op). SNG_EHIP if releasing
 * one of its HIP graph or stream handles failed. */
int sng_batch_plan_destroy(sng_batch_plan *plan);

/* Allocation-free form of sng_dbscan, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Arguments, results and errors are those
 * of sng_dbscan, without workspace: the call uses a static device array of
 * SNG_NOALLOC_SCRATCH_BYTES (32 MiB) that every GPU the library runs on
 * holds until the process ends, and calls no allocating routine. Inputs and
 * outputs are still the caller's. SNG_ERANGE when the workspace sng_dbscan
 * would need (sng_workspace_size with SNG_WS_DIRECT, plus
 * SNG_WS_SIMPLE_GRAPH for the simple-graph mode) exceeds the array, e.g.
 * n = 1e6 points with more than about 200 samples each; SNG_EINVAL with
 * reuse_sample; SNG_EHIP if the array's device address cannot be obtained.
 * All calls on one GPU share its array, which keeps the last call's
 * contents (each call clears what it uses): calls that overlap on one GPU,
 * on any streams or host threads, race and give undefined results, so the
 * caller must order them (e.g. one stream). sng_stats_read cannot reach the
 * array; use sng_dbscan for counters. */
#define SNG_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int sng_dbscan_noalloc(const float *X, int64_t n, int32_t d, int64_t ld, double s, double eps,
                       int32_t min_pts, uint64_t seed, int32_t *labels, uint32_t *degrees,
                       const sng_config *cfg, void *stream);

/* Copies the counters of the last call that used `workspace` (waits for
 * `stream`). Returns SNG_EOVERFLOW if that call's queue overflowed. For a
 * batch workspace, `index` selects the instance; otherwise pass 0. */
int sng_stats_read(const void *workspace, int32_t index, sng_stats *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SNG_H */
