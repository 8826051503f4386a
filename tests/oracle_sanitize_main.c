/* Drives every entry point of the CPU oracle on small seeded inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (host code
 * only). Exits non-zero on a failed check; the sanitizers abort on their own
 * findings. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/sng_oracle.h"

static uint64_t lcg = 0x9E3779B97F4A7C15ull;

static float next_unit(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (float)((lcg >> 40) * (1.0 / 16777216.0));
}

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                              \
        }                                                          \
    } while (0)

static int run_case(int64_t n, int32_t d, int64_t ld, int64_t m)
{
    float *X = (float *)malloc((size_t)(n > 0 ? n : 1) * (size_t)ld * sizeof(float));
    int32_t *labels = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    uint32_t *deg = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    double *sq = (double *)malloc((size_t)(n > 0 ? n : 1) * (size_t)(m > 0 ? m : 1) * sizeof(double));
    uint64_t st[8];
    CHECK(X && labels && deg && sq);
    for (int64_t k = 0; k < n * ld; ++k)
        X[k] = next_unit();
    for (int32_t mode = 0; mode <= 3; ++mode) {
        CHECK(sng_oracle_dbscan(X, n, d, ld, m, 0.3, 3, 7, mode, labels, deg, st) == 0);
        uint64_t sum = 0;
        for (int64_t i = 0; i < n; ++i) {
            sum += deg[i];
            CHECK(labels[i] >= -1 && labels[i] < n);
        }
        if (mode != 2)
            CHECK(sum % 2 == 0);
        for (int32_t kind = 1; kind <= 2; ++kind)
            CHECK(sng_oracle_dbscan_similarity(X, n, d, ld, m, kind, 0.5, 2, 9, mode, labels, NULL,
                                               st) == 0);
    }
    for (int64_t i = 0; i < n; ++i)
        deg[i] = 0;
    CHECK(sng_oracle_degrees_range(X, n, d, ld, m, 0.4, 3, 0, n, deg, st) == 0);
    CHECK(sng_oracle_slot_sqdist(X, n, d, ld, m, 5, 0, n, sq) == 0);
    if (n >= 2) {
        int64_t edges[6] = {0, 1, 1, n - 1, 0, n - 1};
        CHECK(sng_oracle_graph(n, edges, n >= 3 ? 3 : 1, 1, labels, deg, st) == 0);
        CHECK(sng_oracle_dot(X, ld, d, 0, n - 1) == sng_oracle_dot(X, ld, d, n - 1, 0));
        (void)sng_oracle_cosine(X, ld, d, 0, n - 1);
        CHECK(sng_oracle_sqdist(X, ld, d, 0, n - 1) >= 0.0);
    }
    /* invalid arguments are refused before any access */
    CHECK(sng_oracle_dbscan(X, n, 0, ld, m, 0.3, 3, 7, 0, labels, deg, st) == -1);
    CHECK(sng_oracle_dbscan(X, n, d, ld, m, -1.0, 3, 7, 0, labels, deg, st) == -1);
    CHECK(sng_oracle_dbscan(X, n, d, ld, m, 0.3, 3, 7, 4, labels, deg, st) == -1);
    CHECK(sng_oracle_dbscan_similarity(X, n, d, ld, m, 3, 0.5, 2, 9, 0, labels, NULL, st) == -1);
    free(X);
    free(labels);
    free(deg);
    free(sq);
    return 0;
}

int main(void)
{
    uint32_t out[4], key[2] = {1, 2}, ctr[4] = {3, 4, 5, 6};
    uint64_t out64[4], key64[2] = {1, 2}, ctr64[4] = {3, 4, 5, 6};
    sng_oracle_philox4x32_10(ctr, key, out);
    sng_oracle_philox4x64_10(ctr64, key64, out64);
    if (sng_oracle_samples_per_point(0.01, 10000) != 100)
        return 1;
    const int64_t shapes[][4] = {{0, 2, 2, 5}, {1, 1, 1, 9}, {2, 3, 4, 7}, {97, 5, 5, 13},
                                 {300, 2, 3, 40}, {257, 16, 16, 11}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        if (run_case(shapes[s][0], (int32_t)shapes[s][1], shapes[s][2], shapes[s][3]))
            return 1;
    puts("OK");
    return 0;
}
