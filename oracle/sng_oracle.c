/*
 * SNG-DBSCAN CPU oracle -- TEST INFRASTRUCTURE ONLY (see sng_oracle.h).
 *
 * Plain definition of Algorithm 1 (Section 3 of the paper) with the readings
 * listed in sng_oracle.h. Nothing here is tuned: it is meant to be read
 * against the paper. Build: gcc -O2 -fopenmp -ffp-contract=off.
 */
#include "sng_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox-4xW-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11, Section 3.2). One round maps the counter        */
/* (c0,c1,c2,c3) with round key (k0,k1) to                                  */
/*   (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))     */
/* and the key is bumped by the Weyl constants (golden ratio, sqrt(3)-1)    */
/* between rounds. The same macro builds both word widths, so that the      */
/* 64-bit instance (checked against an independent library) pins the round  */
/* structure that the 32-bit instance uses.                                 */
/* ------------------------------------------------------------------------ */

#define PHILOX_ROUNDS 10

#define PHILOX_DEFINE(W, UINT, MULHILO, MA, MB, WA, WB)                              \
    static void philox4x##W##_rounds(UINT c[4], UINT k[2])                          \
    {                                                                                \
        for (int r = 0; r < PHILOX_ROUNDS; ++r) {                                    \
            if (r > 0) {                                                             \
                k[0] += (UINT)(WA);                                                  \
                k[1] += (UINT)(WB);                                                  \
            }                                                                        \
            UINT hi0, lo0, hi1, lo1;                                                 \
            MULHILO((UINT)(MA), c[0], &hi0, &lo0);                                   \
            MULHILO((UINT)(MB), c[2], &hi1, &lo1);                                   \
            UINT n0 = hi1 ^ c[1] ^ k[0];                                             \
            UINT n2 = hi0 ^ c[3] ^ k[1];                                             \
            c[0] = n0;                                                               \
            c[1] = lo1;                                                              \
            c[2] = n2;                                                               \
            c[3] = lo0;                                                              \
        }                                                                            \
    }

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Multipliers and Weyl increments from the SC'11 paper (Table 2 / text). */
PHILOX_DEFINE(32, uint32_t, mulhilo32, 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
PHILOX_DEFINE(64, uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
              0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

void sng_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    philox4x32_rounds(c, k);
    memcpy(out, c, sizeof(c));
}

void sng_oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint64_t k[2] = {key[0], key[1]};
    philox4x64_rounds(c, k);
    memcpy(out, c, sizeof(c));
}

/* ------------------------------------------------------------------------ */
/* Sampling (Algorithm 1: "sample ceil(sn) examples from X_[n]").           */
/* ------------------------------------------------------------------------ */

int64_t sng_oracle_samples_per_point(double s, int64_t n)
{
    if (!(s >= 0.0) || isinf(s) || n < 0)
        return -1;
    double sn = s * (double)n;
    double m = ceil(sn);
    if (m > 17179869184.0) /* t/4 must fit a 32-bit counter word */
        return -1;
    return (int64_t)m;
}

uint32_t sng_oracle_partner(uint64_t seed, int64_t n, int64_t i, int64_t t)
{
    uint32_t ctr[4] = {(uint32_t)(t / 4), (uint32_t)i, 0u, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    sng_oracle_philox4x32_10(ctr, key, w);
    return w[t % 4] % (uint32_t)n;
}

/* ------------------------------------------------------------------------ */
/* Similarity query (Algorithm 1: |x - x'| <= eps), squared, binary64.      */
/* ------------------------------------------------------------------------ */

double sng_oracle_sqdist(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j)
{
    const float *a = X + i * ld;
    const float *b = X + j * ld;
    double acc = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double delta = (double)a[k] - (double)b[k];
        double sq = delta * delta;
        acc = acc + sq;
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Similarity queries other than the distance (Section 1: the method only    */
/* needs a yes/no similarity query per sampled pair, so any similarity      */
/* function can define the edges). An edge joins i and j when their         */
/* similarity is at least tau.                                              */
/* ------------------------------------------------------------------------ */

/* <x_i, x_j> in binary64, products and sums in coordinate order. */
double sng_oracle_dot(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j)
{
    const float *a = X + i * ld;
    const float *b = X + j * ld;
    double acc = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double p = (double)a[k] * (double)b[k];
        acc = acc + p;
    }
    return acc;
}

/* <x_i, x_j> / (sqrt(<x_i, x_i>) * sqrt(<x_j, x_j>)) in binary64; NaN when a
 * row is zero (0 / 0). */
double sng_oracle_cosine(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j)
{
    double ip = sng_oracle_dot(X, ld, d, i, j);
    double ni = sqrt(sng_oracle_dot(X, ld, d, i, i));
    double nj = sqrt(sng_oracle_dot(X, ld, d, j, j));
    double den = ni * nj;
    return ip / den;
}

/* The similarity query of a run: kind 0 is the paper's |x - x'| <= eps
 * (squared, against eps2 = fl64(eps*eps)); kinds 1 and 2 accept when the dot
 * product or the cosine is >= tau. */
typedef struct {
    int32_t kind;
    double eps2;
    double tau;
} query;

static int accepted(const float *X, int64_t ld, int32_t d, int64_t i, int64_t j, const query *q)
{
    if (i == j)
        return 0;
    switch (q->kind) {
    case SNG_ORACLE_DOT:
        return sng_oracle_dot(X, ld, d, i, j) >= q->tau; /* false for NaN */
    case SNG_ORACLE_COSINE:
        return sng_oracle_cosine(X, ld, d, i, j) >= q->tau;
    default:
        return sng_oracle_sqdist(X, ld, d, i, j) <= q->eps2;
    }
}

static query distance_query(double eps)
{
    query q = {0, eps * eps, 0.0};
    return q;
}

/* ------------------------------------------------------------------------ */
/* Growable per-thread list of accepted pairs (the edge set A of G).        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t *v;
    int64_t len, cap;
    int failed;
} pairlist;

static void pl_push(pairlist *p, int64_t a, int64_t b)
{
    if (p->failed)
        return;
    if (p->len + 2 > p->cap) {
        int64_t nc = p->cap ? 2 * p->cap : 1024;
        int64_t *nv = (int64_t *)realloc(p->v, (size_t)nc * sizeof(int64_t));
        if (!nv) {
            p->failed = 1;
            return;
        }
        p->v = nv;
        p->cap = nc;
    }
    p->v[p->len++] = a;
    p->v[p->len++] = b;
}

static int valid_points(const float *X, int64_t n, int32_t d, int64_t ld)
{
    if (n < 0 || n > 2147483647LL || d < 1 || ld < d)
        return 0;
    if (n > 0 && !X)
        return 0;
    return 1;
}

static int valid_eps(double eps)
{
    return eps >= 0.0 && !isinf(eps);
}

/* Sampling step for sources [i0,i1): degrees (atomic integer adds, so the
 * result does not depend on thread order) and, optionally, the accepted
 * pairs gathered into *out (order irrelevant to everything downstream). */
static int sample_graph(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                        const query *q, uint64_t seed, int64_t i0, int64_t i1, uint32_t *deg,
                        uint64_t *stats, pairlist *out, int symmetrised)
{
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    pairlist *lists = (pairlist *)calloc((size_t)nthreads, sizeof(pairlist));
    if (!lists)
        return -3;
    uint64_t self_total = 0, acc_total = 0;
#pragma omp parallel reduction(+ : self_total, acc_total)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = i0; i < i1; ++i) {
            for (int64_t t = 0; t < m; ++t) {
                int64_t j = (int64_t)sng_oracle_partner(seed, n, i, t);
                if (j == i) {
                    self_total++;
                    continue;
                }
                if (accepted(X, ld, d, i, j, q)) {
                    acc_total++;
#pragma omp atomic
                    deg[i]++;
                    if (symmetrised) {
#pragma omp atomic
                        deg[j]++;
                    }
                    if (out)
                        pl_push(&lists[tid], i, j);
                }
            }
        }
    }
    int rc = 0;
    if (out) {
        int64_t total = 0;
        for (int k = 0; k < nthreads; ++k) {
            if (lists[k].failed)
                rc = -3;
            total += lists[k].len;
        }
        if (rc == 0) {
            out->v = (int64_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int64_t));
            out->len = out->cap = total;
            if (!out->v)
                rc = -3;
            int64_t pos = 0;
            for (int k = 0; k < nthreads && rc == 0; ++k) {
                if (lists[k].len)
                    memcpy(out->v + pos, lists[k].v, (size_t)lists[k].len * sizeof(int64_t));
                pos += lists[k].len;
            }
        }
    }
    for (int k = 0; k < nthreads; ++k)
        free(lists[k].v);
    free(lists);
    if (stats) {
        stats[0] += (uint64_t)(i1 - i0) * (uint64_t)m;
        stats[1] += self_total;
        stats[2] += acc_total;
    }
    return rc;
}

int sng_oracle_degrees_range(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                             double eps, uint64_t seed, int64_t i0, int64_t i1,
                             uint32_t *deg, uint64_t *stats)
{
    if (!valid_points(X, n, d, ld) || !valid_eps(eps) || m < 0 || i0 < 0 || i1 > n || i0 > i1 ||
        !deg)
        return -1;
    if (n == 0)
        return 0;
    const query q = distance_query(eps);
    return sample_graph(X, n, d, ld, m, &q, seed, i0, i1, deg, stats, NULL, 1);
}

int sng_oracle_slot_sqdist(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                           uint64_t seed, int64_t i0, int64_t i1, double *out)
{
    if (!valid_points(X, n, d, ld) || m < 0 || i0 < 0 || i1 > n || i0 > i1 || !out)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = i0; i < i1; ++i) {
        for (int64_t t = 0; t < m; ++t) {
            int64_t j = (int64_t)sng_oracle_partner(seed, n, i, t);
            out[(i - i0) * m + t] = (j == i) ? -1.0 : sng_oracle_sqdist(X, ld, d, i, j);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Post-processing (Algorithm 1, last three steps): core points, connected   */
/* components of the core-induced subgraph, border assignment.              */
/* ------------------------------------------------------------------------ */

static int64_t uf_find(int64_t *parent, int64_t x)
{
    int64_t r = x;
    while (parent[r] != r)
        r = parent[r];
    while (parent[x] != r) { /* path compression */
        int64_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

static void uf_union(int64_t *parent, int64_t a, int64_t b)
{
    int64_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb)
        return;
    /* keep the smaller index as the root, so each root is its component's
     * minimum member */
    if (ra < rb)
        parent[rb] = ra;
    else
        parent[ra] = rb;
}

static int postprocess(int64_t n, const pairlist *A, const uint32_t *deg, int32_t min_pts,
                       int32_t *labels, uint64_t *stats)
{
    char *core = (char *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *parent = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *best = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!core || !parent || !best) {
        free(core);
        free(parent);
        free(best);
        return -3;
    }
    int64_t n_core = 0;
    for (int64_t i = 0; i < n; ++i) {
        core[i] = (int64_t)deg[i] >= (int64_t)min_pts;
        n_core += core[i];
        parent[i] = i;
        best[i] = -1;
    }
    /* components K_1..K_l of the subgraph induced by core vertices */
    for (int64_t e = 0; e < A->len; e += 2) {
        int64_t a = A->v[e], b = A->v[e + 1];
        if (core[a] && core[b])
            uf_union(parent, a, b);
    }
    /* border points: smallest-index core neighbour */
    for (int64_t e = 0; e < A->len; e += 2) {
        int64_t a = A->v[e], b = A->v[e + 1];
        if (core[a] && !core[b] && (best[b] < 0 || a < best[b]))
            best[b] = a;
        if (core[b] && !core[a] && (best[a] < 0 || b < best[a]))
            best[a] = b;
    }
    int64_t n_clusters = 0, n_noise = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (core[i]) {
            int64_t r = uf_find(parent, i);
            labels[i] = (int32_t)r;
            n_clusters += (r == i);
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!core[i]) {
            labels[i] = best[i] < 0 ? -1 : labels[best[i]];
            n_noise += (best[i] < 0);
        }
    }
    if (stats) {
        stats[3] = (uint64_t)n_core;
        stats[4] = (uint64_t)n_clusters;
        stats[5] = (uint64_t)n_noise;
    }
    free(core);
    free(parent);
    free(best);
    return 0;
}

/* Simple-graph degrees: each distinct pair {a, b} of the accepted list
 * counts once for both endpoints, however many slots sampled it, in either
 * direction (the graph G of Algorithm 1 read as a simple graph). */
static int cmp_i64(const void *x, const void *y)
{
    const int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

static int simple_degrees(int64_t n, const pairlist *A, uint32_t *deg)
{
    const int64_t k = A->len / 2;
    int64_t *keys = (int64_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int64_t));
    if (!keys)
        return -3;
    for (int64_t e = 0; e < k; ++e) {
        int64_t a = A->v[2 * e], b = A->v[2 * e + 1];
        keys[e] = a < b ? a * n + b : b * n + a;
    }
    qsort(keys, (size_t)k, sizeof(int64_t), cmp_i64);
    memset(deg, 0, (size_t)n * sizeof(uint32_t));
    for (int64_t e = 0; e < k; ++e) {
        if (e > 0 && keys[e] == keys[e - 1])
            continue;
        deg[keys[e] / n]++;
        deg[keys[e] % n]++;
    }
    free(keys);
    return 0;
}

/* The whole method for one similarity query (validated by the callers). */
static int run_method(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                      const query *q, int32_t min_pts, uint64_t seed, int32_t mode,
                      int32_t *labels, uint32_t *deg, uint64_t *stats)
{
    if (mode != 1 && (m > 17179869184LL || (m > 0 && n > INT64_MAX / m)))
        return -2;
    uint64_t local[8] = {0};
    uint32_t *dg = deg ? deg : (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    if (!dg)
        return -3;
    memset(dg, 0, (size_t)n * sizeof(uint32_t));
    pairlist A = {0};
    int rc = 0;
    if (mode != 1) {
        /* mode 2: a point's degree counts only its own accepted samples (the
         * neighbour count of Lemma 2's proof); the graph is the same. */
        if (n > 0)
            rc = sample_graph(X, n, d, ld, m, q, seed, 0, n, dg, local, &A, mode != 2);
        /* mode 3: the degree of the simple graph instead of the multigraph */
        if (rc == 0 && mode == 3)
            rc = simple_degrees(n, &A, dg);
    } else {
        /* exhaustive: the full neighbourhood graph of classical DBSCAN */
        for (int64_t i = 0; i < n && rc == 0; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                if (accepted(X, ld, d, i, j, q)) {
                    dg[i]++;
                    dg[j]++;
                    local[2]++;
                    pl_push(&A, i, j);
                }
        local[0] = (uint64_t)(n * (n - 1) / 2);
        if (A.failed)
            rc = -3;
    }
    if (rc == 0)
        rc = postprocess(n, &A, dg, min_pts, labels, local);
    free(A.v);
    if (!deg)
        free(dg);
    if (rc == 0 && stats)
        memcpy(stats, local, sizeof(local));
    return rc;
}

int sng_oracle_dbscan(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                      double eps, int32_t min_pts, uint64_t seed, int32_t mode,
                      int32_t *labels, uint32_t *deg, uint64_t *stats)
{
    if (!valid_points(X, n, d, ld) || !valid_eps(eps) || mode < 0 || mode > 3 ||
        (n > 0 && !labels) || (mode != 1 && m < 0))
        return -1;
    const query q = distance_query(eps);
    return run_method(X, n, d, ld, m, &q, min_pts, seed, mode, labels, deg, stats);
}

int sng_oracle_dbscan_similarity(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                                 int32_t kind, double tau, int32_t min_pts, uint64_t seed,
                                 int32_t mode, int32_t *labels, uint32_t *deg, uint64_t *stats)
{
    if (!valid_points(X, n, d, ld) || (kind != SNG_ORACLE_DOT && kind != SNG_ORACLE_COSINE) ||
        isnan(tau) || isinf(tau) || mode < 0 || mode > 3 || (n > 0 && !labels) ||
        (mode != 1 && m < 0))
        return -1;
    const query q = {kind, 0.0, tau};
    return run_method(X, n, d, ld, m, &q, min_pts, seed, mode, labels, deg, stats);
}

/* A grid of (eps, MinPts) pairs (Section 5 tunes eps over a grid of values),
 * each solved as by sng_oracle_dbscan in mode 0 or 2. The sampling step runs
 * once, at the largest eps of the grid, and keeps its accepted pairs; pair
 * (i,j) is an edge at eps[k] iff D(i,j) <= fl64(eps[k]*eps[k]), the single
 * run's own test, recomputed here per pair. Every edge at eps[k] is among
 * the kept pairs because rounding eps*eps is monotone in eps. */
int sng_oracle_sweep(const float *X, int64_t n, int32_t d, int64_t ld, int64_t m,
                     const double *eps, int32_t n_eps, const int32_t *min_pts, int32_t n_minpts,
                     uint64_t seed, int32_t mode, int32_t *labels, uint32_t *deg, uint64_t *stats)
{
    if (!valid_points(X, n, d, ld) || m < 0 || n_eps < 1 || n_minpts < 1 || !eps || !min_pts ||
        (mode != 0 && mode != 2) || (n > 0 && !labels))
        return -1;
    double eps_max = 0.0;
    for (int32_t k = 0; k < n_eps; ++k) {
        if (!valid_eps(eps[k]))
            return -1;
        if (eps[k] > eps_max)
            eps_max = eps[k];
    }
    if (m > 17179869184LL || (m > 0 && n > INT64_MAX / m))
        return -2;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    uint32_t *dg = (uint32_t *)calloc(nn, sizeof(uint32_t));
    uint32_t *dk = (uint32_t *)malloc(nn * sizeof(uint32_t));
    pairlist A = {0}, Ak = {0};
    uint64_t base[8] = {0};
    int rc = (dg && dk) ? 0 : -3;
    const query qmax = distance_query(eps_max);
    if (rc == 0 && n > 0)
        rc = sample_graph(X, n, d, ld, m, &qmax, seed, 0, n, dg, base, &A, 1);
    if (rc == 0) {
        Ak.v = (int64_t *)malloc((size_t)(A.len > 0 ? A.len : 1) * sizeof(int64_t));
        if (!Ak.v)
            rc = -3;
    }
    for (int32_t k = 0; k < n_eps && rc == 0; ++k) {
        const query q = distance_query(eps[k]);
        Ak.len = 0;
        memset(dk, 0, nn * sizeof(uint32_t));
        for (int64_t e = 0; e < A.len; e += 2) {
            const int64_t a = A.v[e], b = A.v[e + 1]; /* a is the sampling point */
            if (!accepted(X, ld, d, a, b, &q))
                continue;
            Ak.v[Ak.len++] = a;
            Ak.v[Ak.len++] = b;
            dk[a]++;
            if (mode != 2)
                dk[b]++;
        }
        if (deg && n > 0)
            memcpy(deg + (size_t)k * (size_t)n, dk, (size_t)n * sizeof(uint32_t));
        for (int32_t p = 0; p < n_minpts && rc == 0; ++p) {
            uint64_t local[8] = {base[0], base[1], (uint64_t)(Ak.len / 2), 0, 0, 0, 0, 0};
            rc = postprocess(n, &Ak, dk, min_pts[p],
                             labels + ((size_t)p * (size_t)n_eps + (size_t)k) * (size_t)n, local);
            if (rc == 0 && stats)
                memcpy(stats + ((size_t)p * (size_t)n_eps + (size_t)k) * 8, local, sizeof(local));
        }
    }
    free(A.v);
    free(Ak.v);
    free(dg);
    free(dk);
    return rc;
}

int sng_oracle_graph(int64_t n, const int64_t *edges, int64_t n_edges, int32_t min_pts,
                     int32_t *labels, uint32_t *deg, uint64_t *stats)
{
    if (n < 0 || n > 2147483647LL || n_edges < 0 || (n_edges > 0 && !edges) || (n > 0 && !labels))
        return -1;
    for (int64_t e = 0; e < n_edges; ++e) {
        int64_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b)
            return -1;
    }
    uint64_t local[8] = {0};
    uint32_t *dg = deg ? deg : (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    if (!dg)
        return -3;
    memset(dg, 0, (size_t)n * sizeof(uint32_t));
    for (int64_t e = 0; e < n_edges; ++e) {
        dg[edges[2 * e]]++;
        dg[edges[2 * e + 1]]++;
    }
    pairlist A = {(int64_t *)edges, 2 * n_edges, 2 * n_edges, 0};
    local[0] = (uint64_t)n_edges;
    local[2] = (uint64_t)n_edges;
    int rc = postprocess(n, &A, dg, min_pts, labels, local);
    if (!deg)
        free(dg);
    if (rc == 0 && stats)
        memcpy(stats, local, sizeof(local));
    return rc;
}
