/*
 * SNG-DBSCAN CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct host implementation of what the SNG-DBSCAN
 * hot path computes (Jiang, Jang, Lacki, "Faster DBSCAN via subsampled
 * similarity queries", NeurIPS 2020; Algorithm 1 in Section 3). Only the test
 * suite, the package smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or constant with the GPU library.
 *
 * All pointers are host pointers. Floating-point work is binary64, evaluated
 * in sequential coordinate order, round-to-nearest-even, without contraction
 * (the library is built with -ffp-contract=off).
 *
 * Readings of the paper that fix what Algorithm 1 leaves open (all binding):
 *  - sampling is with replacement over [0,n); sample t of point i is
 *        j = Philox4x32-10(ctr = (t/4, i, 0, 0), key = (seed mod 2^32,
 *            seed / 2^32)) word (t mod 4), reduced mod n,
 *    for t < m = ceil(fl64(s*n));
 *  - a self-sample (j == i) adds no edge;
 *  - the graph is a symmetrised multigraph: every accepted sample adds one to
 *    the degree of both endpoints, repeated samples count again;
 *  - a pair is an edge iff D(i,j) <= fl64(eps*eps), D the squared Euclidean
 *    distance as described above (inclusive, NaN never accepted);
 *  - core iff (int64)degree >= MinPts;
 *  - cluster label = smallest point index of the core component; a non-core
 *    point takes the label of its smallest-index core neighbour, else -1.
 *
 * Return codes: 0 on success, -1 on invalid arguments (nothing written),
 * -2 on a size out of range, -3 on allocation failure.
 */
#ifndef SNG_ORACLE_H
#define SNG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox-4x32 and Philox-4x64 with 10 rounds (Salmon et al., SC'11, Sec. 3). */
void sng_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void sng_oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* m = ceil(fl64(s*n)); -1 if s is negative, NaN or infinite, or n < 0. */
int64_t sng_oracle_samples_per_point(double s, int64_t n);

/* The t-th sampled partner of point i (Algorithm 1, sampling step). */
uint32_t sng_oracle_partner(uint64_t seed, int64_t n, int64_t i, int64_t t);

/* D(i,j): binary64 squared distance of rows i and j of X (row stride ld). */
double sng_oracle_sqdist(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j);

/* Similarity functions other than the distance (Section 1: the method needs
 * only a similarity query per sampled pair). An edge joins i and j when the
 * similarity is >= tau (inclusive, NaN never accepted).
 *   SNG_ORACLE_DOT:    <x_i, x_j>, products and sums in binary64 in
 *                      coordinate order;
 *   SNG_ORACLE_COSINE: <x_i, x_j> / (sqrt(<x_i, x_i>) * sqrt(<x_j, x_j>)),
 *                      each part as for DOT, correctly rounded sqrt, product
 *                      and quotient; a zero row gives NaN, so no edge. */
#define SNG_ORACLE_DOT 1
#define SNG_ORACLE_COSINE 2
double sng_oracle_dot(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j);
double sng_oracle_cosine(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j);

/* stats[0..7] = slots, self_pairs, accepted, n_core, n_clusters, n_noise,
 * 0, 0.  Any of stats/deg may be NULL where noted. */

/* Sampling step over sources [i0, i1): adds the symmetrised degrees into
 * deg[n] (which the caller zeroes) and counts slots/self/accepted into
 * stats[0..2] (added). Uses OpenMP threads. */
int sng_oracle_degrees_range(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                             double eps, uint64_t seed, int64_t i0, int64_t i1,
                             uint32_t *deg, uint64_t *stats);

/* D for every slot of sources [i0,i1): out[(i-i0)*m + t]; -1.0 for a
 * self-sample. */
int sng_oracle_slot_sqdist(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                           uint64_t seed, int64_t i0, int64_t i1, double *out);

/* Whole method. mode 0: Philox-sampled graph with m samples per point.
 * mode 1: exhaustive graph (every unordered pair i<j once; m ignored), i.e.
 * full DBSCAN on the same post-processing. mode 2: the sampled graph of mode
 * 0, but a point's degree (and so its core test) counts only its own
 * accepted samples (Lemma 2, Section 4.1, and its proof); components and
 * borders still use every accepted pair. mode 3: the sampled graph of mode
 * 0 read as a simple graph: a point's degree is its number of distinct
 * accepted neighbours, a pair sampled several times (by either endpoint)
 * counting once. labels[n] and deg[n] are written; deg may be NULL. */
int sng_oracle_dbscan(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                      double eps, int32_t min_pts, uint64_t seed, int32_t mode,
                      int32_t *labels, uint32_t *deg, uint64_t *stats);

/* sng_oracle_dbscan with the similarity query `kind` (SNG_ORACLE_DOT or
 * SNG_ORACLE_COSINE) against a finite tau instead of the distance against
 * eps; modes, outputs and everything after the query as there. */
int sng_oracle_dbscan_similarity(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                                 int32_t kind, double tau, int32_t min_pts, uint64_t seed,
                                 int32_t mode, int32_t *labels, uint32_t *deg, uint64_t *stats);

/* Every (eps[k], min_pts[p]) pair of a grid (Section 5 tunes eps over a
 * grid): labels[(p*n_eps + k)*n + i] and deg[k*n + i] (deg may be NULL) equal
 * those of sng_oracle_dbscan(eps[k], min_pts[p]) in `mode` (0 or 2); stats,
 * if not NULL, holds 8 values per (p, k) in the same order. eps in any
 * order, each finite and >= 0. */
int sng_oracle_sweep(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                     const double *eps, int32_t n_eps, const int32_t *min_pts, int32_t n_minpts,
                     uint64_t seed, int32_t mode, int32_t *labels, uint32_t *deg,
                     uint64_t *stats);

/* Post-processing only, on an explicit accepted-pair list edges[2*k],
 * edges[2*k+1] (each pair counted once per occurrence, self-pairs rejected
 * with -1). */
int sng_oracle_graph(int64_t n, const int64_t *edges, int64_t n_edges, int32_t min_pts,
                     int32_t *labels, uint32_t *deg, uint64_t *stats);

#ifdef __cplusplus
}
#endif
#endif
