/*
 * oracle_driver.c -- runs the FP64 oracle's core cases in one process so that
 * the oracle can be built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py).  Test code only: it declares the oracle's
 * entry points itself and checks a few identities of each result, so a run
 * that is clean under the sanitizers is also a sane one.
 * Exit status 0 and the line "driver ok" mean every case ran and held.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double lo, hi;
    int32_t count, half_open;
} axis_t;

typedef struct {
    double fs;
    int32_t n, pad;
    axis_t ax[4];
} grid_t;

typedef struct {
    int32_t samples, levels, topk, pad;
    int32_t radius[4];
    double step[8][4];
} lem_t;

int64_t oracle_grid_size(const grid_t* g);
void oracle_grid_theta(const grid_t* g, int64_t i, double theta[4]);
double oracle_atom_unit(double fs, int32_t n, const double theta[4], double* g);
void oracle_correlate(const grid_t* grid, const double* r, int64_t begin, int64_t count, double* p);
void oracle_correlate_many(const grid_t* grid, int32_t m, const double* r, int64_t begin, int64_t count, double* p);
void oracle_correlate_complex_many(const grid_t* grid, int32_t m, const double* r, int64_t begin, int64_t count,
                                   double* p);
int64_t oracle_argmax(const double* p, int64_t k, double* gap);
double oracle_objective(double fs, int32_t n, const double theta[4], const double* r, double grad[4], double* dr);
void oracle_refine_box(const grid_t* grid, double step[4], double lo[4], double hi[4]);
int oracle_refine(double fs, int32_t n, const double* r, const double theta0[4], const double step[4],
                  const double lo[4], const double hi[4], int32_t steps, double theta_out[4], double* j_out);
void oracle_decompose(const grid_t* grid, int32_t batch, const double* s, int32_t order, int32_t refine_steps,
                      double* resid, double* approx, double* theta, double* coef, int64_t* index, double* energy,
                      double* gap, int32_t* flags);
void oracle_decompose_prior(const grid_t* grid, int32_t batch, const double* s, int32_t order, int32_t refine_steps,
                            double* resid, double* approx, double* theta, double* coef, int64_t* index,
                            double* energy, int32_t* flags);
void oracle_decompose_complex(const grid_t* grid, int32_t batch, const double* s, int32_t order,
                              int32_t refine_steps, double* resid, double* approx, double* theta, double* coef_re,
                              double* coef_im, int64_t* index, double* energy, double* gap, int32_t* flags);
void oracle_lem_decompose(const grid_t* grid, const lem_t* cfg, int32_t batch, const double* s, const double* lhs,
                          int32_t order, int32_t refine_steps, double* resid, double* approx, double* theta,
                          double* coef, double* energy, int32_t* flags);
void oracle_reconstruct(double fs, int32_t n, int32_t order, const double* theta, const double* coef, double* out);

static int failures = 0;
#define CHECK(cond, what)                                      \
    do {                                                       \
        if (!(cond)) {                                         \
            fprintf(stderr, "driver check failed: %s\n", what); \
            ++failures;                                        \
        }                                                      \
    } while (0)

/* deterministic uniforms (a 64-bit linear congruential generator) */
static uint64_t lcg = 0x2607166290ULL;
static double uniform(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}
static double normal(void) {
    double u = uniform(), v = uniform();
    return sqrt(-2.0 * log(u + 1e-300)) * cos(6.283185307179586 * v);
}

int main(void) {
    enum { B = 2, N = 96, ORDER = 4 };
    grid_t g = {64.0, N, 0, {{0.0, 1.5, 6, 1}, {2.0, 20.0, 5, 0}, {-4.0, 4.0, 3, 0}, {-2.5, -0.5, 4, 0}}};
    const int64_t K = oracle_grid_size(&g);
    double* s = malloc(sizeof(double) * B * N);
    for (int i = 0; i < B * N; ++i) s[i] = normal();

    /* correlation: single and batched rows agree; arg-max and gap */
    double* p = malloc(sizeof(double) * K);
    double* pm = malloc(sizeof(double) * B * K);
    oracle_correlate(&g, s, 0, K, p);
    oracle_correlate_many(&g, B, s, 0, K, pm);
    CHECK(memcmp(p, pm, sizeof(double) * K) == 0, "correlate_many row 0");
    double gap = -1.0;
    int64_t best = oracle_argmax(p, K, &gap);
    CHECK(best >= 0 && best < K && gap >= 0.0 && gap <= 1.0, "argmax");
    oracle_correlate_complex_many(&g, B, s, 0, K, pm);
    for (int64_t j = 0; j < B * K; ++j) CHECK(pm[j] >= 0.0 && isfinite(pm[j]), "complex scores are magnitudes");

    /* objective, gradient, dJ/dr, refinement */
    double th0[4], grad[4], step[4], lo[4], hi[4], th[4], J = 0.0;
    double* dr = malloc(sizeof(double) * N);
    oracle_grid_theta(&g, best, th0);
    double J0 = oracle_objective(g.fs, N, th0, s, grad, dr);
    CHECK(J0 > 0.0, "objective");
    oracle_refine_box(&g, step, lo, hi);
    oracle_refine(g.fs, N, s, th0, step, lo, hi, 30, th, &J);
    CHECK(J >= J0, "refinement does not lower J");

    /* decompositions: residue-based, prior, complex, LEM; reconstruction */
    double *resid = malloc(sizeof(double) * B * N), *approx = malloc(sizeof(double) * B * N);
    double *theta = malloc(sizeof(double) * B * ORDER * 4), *coef = malloc(sizeof(double) * B * ORDER);
    double *coef2 = malloc(sizeof(double) * B * ORDER), *energy = malloc(sizeof(double) * B * (ORDER + 1));
    double* gaps = malloc(sizeof(double) * B * ORDER);
    int64_t* index = malloc(sizeof(int64_t) * B * ORDER);
    int32_t flags[B];
    double* rec = malloc(sizeof(double) * N);

    oracle_decompose(&g, B, s, ORDER, 30, resid, approx, theta, coef, index, energy, gaps, flags);
    for (int b = 0; b < B; ++b) {
        for (int k = 0; k < ORDER; ++k)
            CHECK(energy[b * (ORDER + 1) + k + 1] <= energy[b * (ORDER + 1) + k] * (1 + 1e-12), "monotone energy");
        oracle_reconstruct(g.fs, N, ORDER, theta + (size_t)b * ORDER * 4, coef + (size_t)b * ORDER, rec);
        for (int t = 0; t < N; ++t) CHECK(fabs(rec[t] - approx[b * N + t]) <= 1e-12 * 10.0, "reconstruct");
    }
    oracle_decompose_prior(&g, B, s, ORDER, 10, resid, approx, theta, coef, index, energy, flags);
    oracle_decompose_complex(&g, B, s, ORDER, 10, resid, approx, theta, coef, coef2, index, energy, gaps, flags);
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < ORDER; ++k)
            CHECK(energy[b * (ORDER + 1) + k + 1] <= energy[b * (ORDER + 1) + k] * (1 + 1e-12), "complex energy");

    lem_t cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.samples = 9;
    cfg.levels = 2;
    cfg.topk = 3;
    cfg.radius[0] = 1;
    cfg.radius[1] = 2;
    cfg.radius[2] = 1;
    cfg.radius[3] = 1;
    for (int l = 0; l <= 2; ++l)
        for (int d = 0; d < 4; ++d) cfg.step[l][d] = step[d] / (double)(1 << l);
    double* lhs = malloc(sizeof(double) * B * ORDER * cfg.samples * 4);
    for (int i = 0; i < B * ORDER * cfg.samples * 4; ++i) lhs[i] = uniform();
    oracle_lem_decompose(&g, &cfg, B, s, lhs, ORDER, 20, resid, approx, theta, coef, energy, flags);
    for (int b = 0; b < B; ++b)
        for (int t = 0; t < N; ++t)
            CHECK(fabs(resid[b * N + t] + approx[b * N + t] - s[b * N + t]) <= 1e-12 * 10.0, "LEM a + r = s");

    free(lhs);
    free(rec);
    free(index);
    free(gaps);
    free(energy);
    free(coef2);
    free(coef);
    free(theta);
    free(approx);
    free(resid);
    free(dr);
    free(pm);
    free(p);
    free(s);
    if (failures) return 1;
    printf("driver ok\n");
    return 0;
}
