/*
 * Runs every entry point of the CPU oracle (oracle/oi_oracle.c) on small
 * generated graphs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exits 0 when every
 * call returns its expected status; the sanitizers abort on any memory or
 * undefined-behaviour error.  Test infrastructure only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double mu, mu1, ups, ups1, ups2;
    uint64_t T1, h1, nsigma, D_lo, D_hi, T, hT, drawn_x, drawn_xp;
    int32_t gsra_only, early;
} rsa_result;

void oo_set_stage1_skip(int64_t min_l);
void oo_set_stage1_skip_cost(double cost);
void oo_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int oo_sample_fixed(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t,
                    uint32_t, uint32_t, uint32_t, uint64_t, uint64_t, uint32_t *, uint64_t *, uint64_t *, double *,
                    int);
int oo_mc_fixed(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, uint32_t,
                uint32_t, uint32_t, uint64_t, uint64_t, uint32_t *, uint64_t *, uint64_t *, int64_t *, int);
int oo_lt_fixed(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, uint32_t,
                uint32_t, uint32_t, uint64_t, uint64_t, uint32_t *, uint64_t *, uint64_t *, int64_t *, int);
int oo_stage1(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, int64_t,
              int64_t *, double *, int32_t *, double *, double *, uint64_t *, int64_t *);
int oo_selection(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, uint32_t,
                 uint32_t, uint32_t, uint64_t, uint64_t, int64_t *);
int oo_rsa_arrays(const uint32_t *, uint64_t, const uint32_t *, uint64_t, double, double, double, double, double,
                  double, rsa_result *);
int oo_rsa_plan(double, double, double, double, double, double, uint64_t, const uint64_t *, const uint64_t *,
                const uint64_t *, const uint64_t *, uint64_t *, uint64_t *, double *);
int oo_gsra_array(const uint32_t *, uint64_t, double, double, double, double, double, double, double *, uint64_t *,
                  uint64_t *, double *);
int oo_estimate(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, double,
                double, int, uint32_t, uint32_t, double *, double *, double *, int64_t *, rsa_result *);
int oo_estimate_lt(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t,
                   double, double, uint32_t, uint32_t, double *, double *, int64_t *, rsa_result *);
int oo_exact(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, double *,
             double *, double *);
int oo_backward(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *, int64_t, uint32_t,
                uint32_t, uint64_t, uint64_t, double *, double *, uint64_t *, double *, int);

static int fails = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

/* a random graph without self-loops: every node gets `deg` out-edges to
 * distinct targets, sorted; probabilities in [0.02, 0.5) (LT weights scaled
 * below so that in-weights sum to at most 1) */
static void make_graph(int64_t n, int64_t deg, uint64_t seed, int64_t **rp, int32_t **col, float **p)
{
    int64_t m = n * deg;
    *rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
    *col = malloc(sizeof(int32_t) * (size_t)m);
    *p = malloc(sizeof(float) * (size_t)m);
    uint64_t x = seed;
    for (int64_t u = 0; u < n; ++u) {
        (*rp)[u] = u * deg;
        for (int64_t k = 0; k < deg; ++k) {
            int32_t v;
            int dup;
            do {
                x = x * 6364136223846793005ull + 1442695040888963407ull;
                v = (int32_t)((x >> 33) % (uint64_t)n);
                dup = v == u;
                for (int64_t j = 0; j < k && !dup; ++j) dup = (*col)[u * deg + j] == v;
            } while (dup);
            int64_t j = k;  /* insertion keeps the row sorted */
            while (j > 0 && (*col)[u * deg + j - 1] > v) {
                (*col)[u * deg + j] = (*col)[u * deg + j - 1];
                --j;
            }
            (*col)[u * deg + j] = v;
            (*p)[u * deg + k] = 0.02f + 0.48f * (float)((x >> 11) & 0xFFFF) / 65536.0f;
        }
    }
    (*rp)[n] = m;
}

int main(void)
{
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    oo_philox(ctr, key, out);

    int64_t n = 300, deg = 6, m = n * deg;
    int64_t *rp;
    int32_t *col;
    float *p;
    make_graph(n, deg, 7, &rp, &col, &p);
    int32_t seeds[5] = {3, 40, 40, 150, 299};
    uint32_t *y = malloc(sizeof(uint32_t) * 4096);
    uint64_t *e = malloc(sizeof(uint64_t) * 4096), sums[2];
    double beta0, oi, is;
    int64_t k, l;
    rsa_result r;

    for (int skip = 0; skip < 2; ++skip) {
        oo_set_stage1_skip(skip ? 1 : 4096);
        oo_set_stage1_skip_cost(skip ? 0.0 : 8.0);
        CHECK(oo_sample_fixed(n, m, rp, col, p, seeds, 5, 1, 9, 0, 0, 4096, y, e, sums, &beta0, 3) == 0);
        CHECK(oo_sample_fixed(n, m, rp, col, p, seeds, 1, 1, 9, 1, 1u << 30, 512, y, NULL, sums, &beta0, 1) == 0);
        CHECK(oo_estimate(n, m, rp, col, p, seeds, 5, 0.2, 0.1, 0, 3, 9, &oi, &is, &beta0, &k, &r) == 0);
        CHECK(oo_estimate(n, m, rp, col, p, seeds, 5, 0.2, 0.1, 1, 3, 9, &oi, &is, &beta0, &k, &r) == 0);
        CHECK(oo_estimate(n, m, rp, col, p, seeds, 2, 0.3, 0.1, 1, 3, 9, &oi, &is, &beta0, &k, &r) == 0);
        double *acc = calloc((size_t)m, sizeof(double)), *acc2 = calloc((size_t)m, sizeof(double));
        uint64_t sy;
        CHECK(oo_backward(n, m, rp, col, p, seeds, 5, 2, 9, 0, 2000, acc, acc2, &sy, &beta0, 2) == 0);
        free(acc);
        free(acc2);
    }
    oo_set_stage1_skip(4096);
    oo_set_stage1_skip_cost(8.0);
    CHECK(oo_mc_fixed(n, m, rp, col, p, seeds, 5, 1, 9, 0, 0, 2048, y, e, sums, &k, 2) == 0);
    int64_t sel[64];
    CHECK(oo_selection(n, m, rp, col, p, seeds, 5, 1, 9, 0, 0, 64, sel) == 0);
    int32_t v[64];
    double P[64], cdf[65];
    uint64_t thr[64];
    CHECK(oo_stage1(n, m, rp, col, p, seeds, 2, 64, &l, &beta0, v, P, cdf, thr, &k) == 0);
    /* LT weights: divide by the in-degree bound so that in-weights sum below 1 */
    float *w = malloc(sizeof(float) * (size_t)m);
    for (int64_t i = 0; i < m; ++i) w[i] = p[i] / 40.0f;
    CHECK(oo_lt_fixed(n, m, rp, col, w, seeds, 5, 1, 9, 0, 0, 2048, y, e, sums, &k, 2) == 0);
    CHECK(oo_estimate_lt(n, m, rp, col, w, seeds, 5, 0.3, 0.1, 4, 9, &oi, &is, &k, &r) == 0);
    CHECK(oo_lt_fixed(n, m, rp, col, p, seeds, 5, 1, 9, 0, 0, 16, y, e, sums, &k, 1) != 0); /* weights too large */
    /* stopping rules on arrays, and their error paths */
    uint32_t *xs = malloc(sizeof(uint32_t) * 200000), *xps = malloc(sizeof(uint32_t) * 200000);
    for (int i = 0; i < 200000; ++i) {
        xs[i] = 1 + (uint32_t)(i % 7);
        xps[i] = 1 + (uint32_t)((i * 5) % 7);
    }
    CHECK(oo_rsa_arrays(xs, 200000, xps, 200000, 0.2, 0.1, 1.0, 8.0, 1.0, 0.0, &r) == 0);
    CHECK(oo_rsa_arrays(xs, 4, xps, 4, 0.1, 0.1, 1.0, 8.0, 1.0, 0.0, &r) != 0);
    double mu, ups;
    uint64_t T, h, h1s[3] = {100, 200, 300}, T1s[3] = {50, 60, 70}, ns[3], Ts[3], Dl[3] = {5, 6, 7}, Dh[3] = {0, 0, 0};
    double thr3[3];
    CHECK(oo_gsra_array(xs, 200000, 0.3, 0.1, 1.0, 8.0, 1.0, 0.0, &mu, &T, &h, &ups) == 0);
    CHECK(oo_rsa_plan(0.1, 0.1, 1.0, 8.0, 1.0, 0.0, 3, h1s, T1s, Dl, Dh, ns, Ts, thr3) == 0);
    CHECK(oo_rsa_plan(0.3, 0.1, 1.0, 8.0, 1.0, 0.0, 3, h1s, T1s, Dl, Dh, ns, Ts, thr3) != 0);
    /* invalid inputs */
    int32_t bad[1] = {(int32_t)n};
    CHECK(oo_estimate(n, m, rp, col, p, bad, 1, 0.2, 0.1, 0, 3, 9, &oi, &is, &beta0, &k, &r) != 0);
    CHECK(oo_estimate(n, m, rp, col, p, seeds, 5, 1.5, 0.1, 0, 3, 9, &oi, &is, &beta0, &k, &r) != 0);
    CHECK(oo_sample_fixed(n, m, rp, col, p, seeds, 0, 1, 9, 0, 0, 4, y, e, sums, &beta0, 1) != 0);
    /* exact enumeration on a 12-edge graph */
    int64_t *rp2;
    int32_t *col2;
    float *p2;
    make_graph(6, 2, 11, &rp2, &col2, &p2);
    double ext, dist[7], grad[12];
    CHECK(oo_exact(6, 12, rp2, col2, p2, seeds, 1, &ext, dist, grad) == 0);
    CHECK(oo_exact(6, 12, rp2, col2, p2, bad, 1, &ext, dist, grad) != 0);
    free(rp2); free(col2); free(p2);
    free(w); free(xs); free(xps); free(y); free(e); free(rp); free(col); free(p);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
