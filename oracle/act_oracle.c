/*
 * act_oracle.c -- plain FP64 CPU oracle of the residue-based Adaptive Chirplet
 * Transform (matching pursuit over a unit-norm Gaussian chirplet dictionary).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP library: no header, no helper, no table.  It is deliberately
 * slow and literal: every atom is evaluated sample by sample from Eq. (1),
 * every inner product is a plain left-to-right sum, nothing is blocked, fused
 * or reordered.  OpenMP only splits independent atoms (or independent
 * refinement problems) across threads; it never changes a sum's order.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no -ffast-math).
 *
 * Conventions (readings of the paper, each one fixed here):
 *  - Atom: the real part of Eq. (1), g(t) = exp(-(1/2)((t-t_c)/dt)^2)
 *    * cos(2 pi (c (t-t_c)^2 + f_c (t-t_c))), sampled at t_n = n/fs, with
 *    dt = exp(logdt).  The analytic prefactor of Eq. (1) is dropped because
 *    every atom is rescaled to unit l2 norm before the search (Sec. III-A).
 *  - Parameter vector theta = (t_c [s], f_c [Hz], c [Hz/s], logdt [ln s]).
 *  - Dictionary index i = ((i_tc*n_fc + i_fc)*n_c + i_c)*n_ld + i_ld
 *    (parameter order of Sec. III-A).  Ties in the arg-max go to the lowest i.
 *  - Axis value j: lo + j*((hi-lo)/d), d = count (half-open) or count-1
 *    (closed, whose last value is hi exactly).
 *  - Matching pursuit on the residual (Sec. III-A, Eq. (3)-(4) and Fig.
 *    "simplified residue-driven ACT iteration"): r_0 = s, a_0 = 0; for every
 *    order: coarse arg-max of |<g_i, r_k>|, continuous refinement of theta
 *    from the winner maximising <g(theta), r_k>^2 / <g,g>, coefficient
 *    c_k = <g*, r_k> with the refined unit atom, r_{k+1} = r_k - c_k g*,
 *    a_{k+1} = a_k + c_k g*.  Normalised residue E_k = |r_k|^2/|s|^2 (Eq. (5)).
 *  - Refinement: the paper names BFGS (Sec. III-A) and gives no settings; the
 *    oracle runs the limited-memory BFGS variant specified in
 *    oracle_refine() below in grid-step units, projected onto the grid hull.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559
#define ORACLE_PI 3.141592653589793238462643383280

typedef struct {
    double lo, hi;
    int32_t count, half_open;
} oracle_axis;

typedef struct {
    double fs;
    int32_t n, pad;
    oracle_axis ax[4]; /* t_c, f_c, c, logdt */
} oracle_grid;

enum { ORACLE_FLAG_NONFINITE = 1, ORACLE_FLAG_REFINE_REJECTED = 2, ORACLE_FLAG_LINESEARCH = 4 };

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* numpy.arange counting rule for a (start, stop, step) range (Table
 * "Parameter ranges" gives the dictionary this way). */
int64_t oracle_arange_count(double start, double stop, double step) {
    return (int64_t)ceil((stop - start) / step);
}

double oracle_axis_value(const oracle_axis* a, int32_t j) {
    if (a->count <= 1) return a->lo;
    int32_t d = a->half_open ? a->count : a->count - 1;
    if (!a->half_open && j == a->count - 1) return a->hi;
    return a->lo + (double)j * ((a->hi - a->lo) / (double)d);
}

double oracle_axis_step(const oracle_axis* a) {
    if (a->count <= 1) return 1.0;
    int32_t d = a->half_open ? a->count : a->count - 1;
    return (a->hi - a->lo) / (double)d;
}

int64_t oracle_grid_size(const oracle_grid* g) {
    return (int64_t)g->ax[0].count * g->ax[1].count * g->ax[2].count * g->ax[3].count;
}

void oracle_grid_theta(const oracle_grid* g, int64_t i, double theta[4]) {
    int64_t rem = i;
    int32_t idx[4];
    for (int a = 3; a >= 0; --a) {
        idx[a] = (int32_t)(rem % g->ax[a].count);
        rem /= g->ax[a].count;
    }
    for (int a = 0; a < 4; ++a) theta[a] = oracle_axis_value(&g->ax[a], idx[a]);
}

/* Eq. (1), real part, without the analytic prefactor. */
void oracle_atom_raw(double fs, int32_t n, const double theta[4], double* g) {
    double dt = exp(theta[3]);
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - theta[0];
        double u = tau / dt;
        double env = exp(-0.5 * u * u);
        double phase = TWO_PI * (theta[2] * tau * tau + theta[1] * tau);
        g[k] = env * cos(phase);
    }
}

static double dot(const double* x, const double* y, int32_t n) {
    double s = 0.0;
    for (int32_t k = 0; k < n; ++k) s += x[k] * y[k];
    return s;
}

/* Unit l2 normalisation (Sec. III-A).  Returns the norm of the raw atom; an
 * atom whose raw norm is below 1e-300 is returned as all zeros. */
double oracle_atom_unit(double fs, int32_t n, const double theta[4], double* g) {
    oracle_atom_raw(fs, n, theta, g);
    double nrm = sqrt(dot(g, g, n));
    if (!(nrm >= 1e-300)) {
        for (int32_t k = 0; k < n; ++k) g[k] = 0.0;
        return nrm;
    }
    for (int32_t k = 0; k < n; ++k) g[k] = g[k] / nrm;
    return nrm;
}

/* p_i = <g_i/|g_i|, r> for dictionary atoms [begin, begin+count). */
void oracle_correlate(const oracle_grid* grid, const double* r, int64_t begin, int64_t count,
                      double* p) {
    int32_t n = grid->n;
#pragma omp parallel
    {
        double* g = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < count; ++j) {
            double th[4];
            oracle_grid_theta(grid, begin + j, th);
            oracle_atom_unit(grid->fs, n, th, g);
            p[j] = dot(g, r, n);
        }
        free(g);
    }
}

/* The same scores for m residuals at once: p[t][j] = <g_{begin+j}/|g|, r_t>,
 * r_t = r + t*n, p_t = p + t*count.  Each atom is synthesised once and dotted
 * with every residual; every dot is the same plain left-to-right sum as in
 * oracle_correlate, so row t equals oracle_correlate on r_t bit for bit. */
void oracle_correlate_many(const oracle_grid* grid, int32_t m, const double* r, int64_t begin, int64_t count,
                           double* p) {
    int32_t n = grid->n;
#pragma omp parallel
    {
        double* g = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < count; ++j) {
            double th[4];
            oracle_grid_theta(grid, begin + j, th);
            oracle_atom_unit(grid->fs, n, th, g);
            for (int32_t t = 0; t < m; ++t) p[(size_t)t * (size_t)count + (size_t)j] = dot(g, r + (size_t)t * n, n);
        }
        free(g);
    }
}

/* Unit-atom norms of the dictionary (raw |g_i|), for plan checks. */
void oracle_norms(const oracle_grid* grid, int64_t begin, int64_t count, double* out) {
    int32_t n = grid->n;
#pragma omp parallel
    {
        double* g = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < count; ++j) {
            double th[4];
            oracle_grid_theta(grid, begin + j, th);
            oracle_atom_raw(grid->fs, n, th, g);
            out[j] = sqrt(dot(g, g, n));
        }
        free(g);
    }
}

/* Coarse search: smallest i with |p_i| = max |p| and the relative gap
 * (|p|_(1) - |p|_(2)) / |p|_(1) to the runner-up. */
int64_t oracle_argmax(const double* p, int64_t k, double* gap) {
    int64_t best = 0;
    double b1 = -1.0, b2 = -1.0;
    for (int64_t i = 0; i < k; ++i) {
        double a = fabs(p[i]);
        if (a > b1) {
            b2 = b1;
            b1 = a;
            best = i;
        } else if (a > b2) {
            b2 = a;
        }
    }
    if (gap) *gap = (b1 > 0.0 && b2 >= 0.0) ? (b1 - b2) / b1 : 0.0;
    return best;
}

/* Refinement objective J(theta) = <r,g>^2 / <g,g> (= <r, g/|g|>^2, the
 * square of the |<g(theta), r>| that Sec. III-A maximises) and its closed-form
 * gradient with respect to theta (SI units) and r.  grad / dr may be NULL. */
double oracle_objective(double fs, int32_t n, const double theta[4], const double* r,
                        double grad[4], double* dr) {
    double tc = theta[0], fc = theta[1], c = theta[2];
    double dt = exp(theta[3]);
    double s = 0.0, q = 0.0;
    double rs[4] = {0, 0, 0, 0}, gs[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - tc;
        double u = tau / dt;
        double e = exp(-0.5 * u * u);
        double ph = TWO_PI * (c * tau * tau + fc * tau);
        double co = cos(ph), si = sin(ph);
        double g = e * co;
        double d[4];
        d[0] = e * ((tau / (dt * dt)) * co + TWO_PI * (2.0 * c * tau + fc) * si);
        d[1] = -TWO_PI * tau * e * si;
        d[2] = -TWO_PI * tau * tau * e * si;
        d[3] = (tau * tau / (dt * dt)) * e * co;
        s += r[k] * g;
        q += g * g;
        for (int j = 0; j < 4; ++j) {
            rs[j] += r[k] * d[j];
            gs[j] += g * d[j];
        }
    }
    if (!(q > 0.0)) {
        if (grad) grad[0] = grad[1] = grad[2] = grad[3] = 0.0;
        if (dr) memset(dr, 0, sizeof(double) * (size_t)n);
        return 0.0;
    }
    double J = s * s / q;
    if (grad)
        for (int j = 0; j < 4; ++j) grad[j] = 2.0 * s * rs[j] / q - 2.0 * s * s * gs[j] / (q * q);
    if (dr) {
        double f = 2.0 * s / q;
        for (int32_t k = 0; k < n; ++k) {
            double tau = (double)k / fs - tc;
            double u = tau / dt;
            double e = exp(-0.5 * u * u);
            double ph = TWO_PI * (c * tau * tau + fc * tau);
            dr[k] = f * e * cos(ph);
        }
    }
    return J;
}

/* ---------------------------------------------------------------------------
 * Refinement (Sec. III-A "BFGS refinement"): maximise J from a grid point.
 *
 *   Coordinates u_j = (theta_j - theta0_j) / s_j.  The scale s_j is the
 *   resolution of the unit atom along parameter j at theta0,
 *   s_j = min(step_j, 1/sqrt(G_jj)), G_jj = (|d_j g|^2 - <g,d_j g>^2/|g|^2)/|g|^2
 *   (the squared norm of the part of d_j g orthogonal to g, per unit |g|^2),
 *   so that one unit of u moves the atom by about one radian whatever f_c and
 *   dt are, and never by more than one grid step.  Axes with a single grid
 *   value, or with G_jj <= 0, are frozen.  Minimise f(u) = -J(theta0 + s*u)
 *   on the box of the grid hull with limited-memory BFGS:
 *     memory 8 pairs; H0 = gamma*I, gamma = s'y/y'y of the newest pair
 *     (1 when empty); a pair is stored only if s'y > 1e-12 |s| |y|.
 *     Projected gradient pg: component j is zeroed when u_j sits on a bound
 *     and -g_j points outwards.  Stop when max|pg| <= 1e-11 * max(1, J).
 *     Direction d = two-loop(-g); components pointing out of the box at an
 *     active bound are zeroed; if g'd >= 0, d = -pg.
 *     Step: alpha0 = 1 when the memory holds a pair, else min(1, 1/max|d|);
 *     backtracking (alpha halves, at most 30 trials) on the projected point
 *     u_new = P(u + alpha d), with p = u_new - u, dec = g'p, dnew = g_new'p.
 *     A trial is accepted when dec < 0 and either
 *       Armijo:             f_new <= f + c1 dec (c1 = 1e-4), or
 *       approximate Wolfe:  f_new <= f + 1e-12 |f| and
 *                           0.9 dec <= dnew <= -0.8 dec
 *     (Hager and Zhang's approximate Wolfe conditions with delta = 0.1,
 *     sigma = 0.9), which keeps the iteration converging on the gradient once
 *     FP64 no longer resolves the change of J.  A failed line search ends the
 *     run.
 *   At most `steps` iterations.  The result is accepted only if
 *   J(theta*) >= J(theta0); otherwise theta0 is kept.
 * Returns a flag word (ORACLE_FLAG_*); writes theta* and J(theta*).
 * ------------------------------------------------------------------------- */
#define LBFGS_M 8

double oracle_objective_prior(double fs, int32_t n, const double theta[4], const double* s,
                              double grad[4]);

double oracle_objective_complex(double fs, int32_t n, const double theta[4], const double* r, double grad[4]);

/* mode 0: J of the residue-based ACT; 1: the prior ACT's objective; 2: complex atoms. */
static double refine_eval(double fs, int32_t n, const double* r, const double th0[4],
                          const double h[4], const double u[4], double gu[4], int mode) {
    double th[4], gr[4];
    for (int j = 0; j < 4; ++j) th[j] = th0[j] + h[j] * u[j];
    double J = mode == 1   ? oracle_objective_prior(fs, n, th, r, gr)
               : mode == 2 ? oracle_objective_complex(fs, n, th, r, gr)
                           : oracle_objective(fs, n, th, r, gr, NULL);
    for (int j = 0; j < 4; ++j) gu[j] = -h[j] * gr[j];
    return -J;
}

/* Coordinate scales of the refinement (see above); 0 marks a frozen axis. */
void oracle_refine_scales(double fs, int32_t n, const double theta0[4], const double step[4],
                          const double lo[4], const double hi[4], double h[4]) {
    double tc = theta0[0], fc = theta0[1], c = theta0[2];
    double dt = exp(theta0[3]);
    double q = 0.0, a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - tc;
        double u = tau / dt;
        double e = exp(-0.5 * u * u);
        double ph = TWO_PI * (c * tau * tau + fc * tau);
        double co = cos(ph), si = sin(ph);
        double g = e * co;
        double d[4];
        d[0] = e * ((tau / (dt * dt)) * co + TWO_PI * (2.0 * c * tau + fc) * si);
        d[1] = -TWO_PI * tau * e * si;
        d[2] = -TWO_PI * tau * tau * e * si;
        d[3] = (tau * tau / (dt * dt)) * e * co;
        q += g * g;
        for (int j = 0; j < 4; ++j) {
            a[j] += g * d[j];
            b[j] += d[j] * d[j];
        }
    }
    for (int j = 0; j < 4; ++j) {
        double G = q > 0.0 ? (b[j] - a[j] * a[j] / q) / q : 0.0;
        if (!(hi[j] > lo[j]) || !(G > 0.0)) {
            h[j] = 0.0;
            continue;
        }
        double r = 1.0 / sqrt(G);
        h[j] = r < step[j] ? r : step[j];
    }
}

/* Scales for complex atoms g = E exp(i phi): the metric of the unit complex
 * atom modulo a global phase (the objective |<g_hat, r>|^2 does not see one),
 *   G_jj = (|d_j g|^2 - |<g, d_j g>|^2 / q) / q,  q = <E, E>,
 * with d_j g = (dE_j + i E dphi_j) exp(i phi):
 *   |d_j g|^2 = sum dE_j^2 + E^2 dphi_j^2,
 *   <g, d_j g> = sum E dE_j + i sum E^2 dphi_j. */
void oracle_refine_scales_complex(double fs, int32_t n, const double theta0[4], const double step[4],
                                  const double lo[4], const double hi[4], double h[4]) {
    double tc = theta0[0], fc = theta0[1], c = theta0[2];
    double dt = exp(theta0[3]);
    double q = 0.0, nrm[4] = {0, 0, 0, 0}, re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - tc;
        double u = tau / dt;
        double e = exp(-0.5 * u * u);
        double de[4] = {e * tau / (dt * dt), 0.0, 0.0, e * tau * tau / (dt * dt)};
        double dp[4] = {-TWO_PI * (2.0 * c * tau + fc), TWO_PI * tau, TWO_PI * tau * tau, 0.0};
        q += e * e;
        for (int j = 0; j < 4; ++j) {
            nrm[j] += de[j] * de[j] + e * e * dp[j] * dp[j];
            re[j] += e * de[j];
            im[j] += e * e * dp[j];
        }
    }
    for (int j = 0; j < 4; ++j) {
        double G = q > 0.0 ? (nrm[j] - (re[j] * re[j] + im[j] * im[j]) / q) / q : 0.0;
        if (!(hi[j] > lo[j]) || !(G > 0.0)) {
            h[j] = 0.0;
            continue;
        }
        double r = 1.0 / sqrt(G);
        h[j] = r < step[j] ? r : step[j];
    }
}

static int refine_core(double fs, int32_t n, const double* r, const double theta0[4],
                       const double step[4], const double lo[4], const double hi[4], int32_t steps,
                       double theta_out[4], double* j_out, int mode) {
    double h[4], blo[4], bhi[4], u[4] = {0, 0, 0, 0}, g[4];
    int flags = 0;
    if (mode == 2)
        oracle_refine_scales_complex(fs, n, theta0, step, lo, hi, h);
    else
        oracle_refine_scales(fs, n, theta0, step, lo, hi, h);
    for (int j = 0; j < 4; ++j) {
        blo[j] = h[j] == 0.0 ? 0.0 : (lo[j] - theta0[j]) / h[j];
        bhi[j] = h[j] == 0.0 ? 0.0 : (hi[j] - theta0[j]) / h[j];
    }
    double f = refine_eval(fs, n, r, theta0, h, u, g, mode);
    double f0 = f;
    double S[LBFGS_M][4], Y[LBFGS_M][4], RHO[LBFGS_M];
    int mem = 0, head = 0; /* head = slot of the next insertion */
    for (int it = 0; it < steps; ++it) {
        double pg[4], pgmax = 0.0;
        for (int j = 0; j < 4; ++j) {
            pg[j] = g[j];
            if (u[j] <= blo[j] && g[j] > 0.0) pg[j] = 0.0;
            if (u[j] >= bhi[j] && g[j] < 0.0) pg[j] = 0.0;
            if (fabs(pg[j]) > pgmax) pgmax = fabs(pg[j]);
        }
        double Jc = -f;
        if (pgmax <= 1e-11 * (Jc > 1.0 ? Jc : 1.0)) break;
        /* two-loop recursion, newest pair first */
        double d[4], al[LBFGS_M];
        for (int j = 0; j < 4; ++j) d[j] = -g[j];
        for (int t = 0; t < mem; ++t) {
            int slot = (head - 1 - t + LBFGS_M) % LBFGS_M;
            double a = RHO[slot] * dot(S[slot], d, 4);
            al[t] = a;
            for (int j = 0; j < 4; ++j) d[j] -= a * Y[slot][j];
        }
        double gamma = 1.0;
        if (mem > 0) {
            int newest = (head - 1 + LBFGS_M) % LBFGS_M;
            gamma = dot(S[newest], Y[newest], 4) / dot(Y[newest], Y[newest], 4);
        }
        for (int j = 0; j < 4; ++j) d[j] *= gamma;
        for (int t = mem - 1; t >= 0; --t) {
            int slot = (head - 1 - t + LBFGS_M) % LBFGS_M;
            double b = RHO[slot] * dot(Y[slot], d, 4);
            for (int j = 0; j < 4; ++j) d[j] += (al[t] - b) * S[slot][j];
        }
        for (int j = 0; j < 4; ++j) {
            if (h[j] == 0.0) d[j] = 0.0;
            if (u[j] <= blo[j] && d[j] < 0.0) d[j] = 0.0;
            if (u[j] >= bhi[j] && d[j] > 0.0) d[j] = 0.0;
        }
        if (dot(g, d, 4) >= 0.0)
            for (int j = 0; j < 4; ++j) d[j] = -pg[j];
        double dmax = 0.0;
        for (int j = 0; j < 4; ++j)
            if (fabs(d[j]) > dmax) dmax = fabs(d[j]);
        double alpha = mem > 0 ? 1.0 : (dmax > 1.0 ? 1.0 / dmax : 1.0);
        double un[4], gn[4], fn = 0.0;
        int ok = 0;
        for (int t = 0; t < 30; ++t) {
            for (int j = 0; j < 4; ++j) {
                double v = u[j] + alpha * d[j];
                if (v < blo[j]) v = blo[j];
                if (v > bhi[j]) v = bhi[j];
                un[j] = v;
            }
            fn = refine_eval(fs, n, r, theta0, h, un, gn, mode);
            double dec = 0.0, dnew = 0.0;
            for (int j = 0; j < 4; ++j) {
                dec += g[j] * (un[j] - u[j]);
                dnew += gn[j] * (un[j] - u[j]);
            }
            int armijo = fn <= f + 1e-4 * dec;
            int approx_wolfe = fn <= f + 1e-12 * fabs(f) && dnew >= 0.9 * dec && dnew <= -0.8 * dec;
            if (dec < 0.0 && (armijo || approx_wolfe)) {
                ok = 1;
                break;
            }
            alpha *= 0.5;
        }
        if (!ok) {
            flags |= ORACLE_FLAG_LINESEARCH;
            break;
        }
        double s[4], y[4];
        for (int j = 0; j < 4; ++j) {
            s[j] = un[j] - u[j];
            y[j] = gn[j] - g[j];
        }
        double sy = dot(s, y, 4);
        if (sy > 1e-12 * sqrt(dot(s, s, 4)) * sqrt(dot(y, y, 4))) {
            for (int j = 0; j < 4; ++j) {
                S[head][j] = s[j];
                Y[head][j] = y[j];
            }
            RHO[head] = 1.0 / sy;
            head = (head + 1) % LBFGS_M;
            if (mem < LBFGS_M) ++mem;
        }
        for (int j = 0; j < 4; ++j) {
            u[j] = un[j];
            g[j] = gn[j];
        }
        f = fn;
    }
    if (-f >= -f0) {
        for (int j = 0; j < 4; ++j) theta_out[j] = theta0[j] + h[j] * u[j];
        *j_out = -f;
    } else {
        for (int j = 0; j < 4; ++j) theta_out[j] = theta0[j];
        *j_out = -f0;
        flags |= ORACLE_FLAG_REFINE_REJECTED;
    }
    return flags;
}

int oracle_refine(double fs, int32_t n, const double* r, const double theta0[4],
                  const double step[4], const double lo[4], const double hi[4], int32_t steps,
                  double theta_out[4], double* j_out) {
    return refine_core(fs, n, r, theta0, step, lo, hi, steps, theta_out, j_out, 0);
}

/* Grid-hull box and spacing used by the refinement. */
void oracle_refine_box(const oracle_grid* grid, double step[4], double lo[4], double hi[4]) {
    for (int a = 0; a < 4; ++a) {
        step[a] = oracle_axis_step(&grid->ax[a]);
        lo[a] = oracle_axis_value(&grid->ax[a], 0);
        hi[a] = oracle_axis_value(&grid->ax[a], grid->ax[a].count - 1);
    }
}

/* Many independent refinement problems (one residual and one start each). */
void oracle_refine_many(const oracle_grid* grid, int32_t m, const double* r, const double* theta0,
                        int32_t steps, double* theta_out, double* j_out, int32_t* flags) {
    double step[4], lo[4], hi[4];
    oracle_refine_box(grid, step, lo, hi);
#pragma omp parallel for schedule(dynamic)
    for (int32_t p = 0; p < m; ++p)
        flags[p] = oracle_refine(grid->fs, grid->n, r + (size_t)p * grid->n, theta0 + 4 * p, step,
                                 lo, hi, steps, theta_out + 4 * p, j_out + p);
}

/* ---------------------------------------------------------------------------
 * Residue-based matching pursuit of one or more channels (Sec. III-A).
 * s: [batch][n] signals; resid/approx: [batch][n] outputs (approx may be NULL);
 * theta [batch][order][4], coef [batch][order], index [batch][order],
 * energy [batch][order+1] (energy[0] = |s|^2), gap [batch][order],
 * flags [batch].  refine_steps = 0 keeps the grid parameters (pure MP over the
 * dictionary).
 * ------------------------------------------------------------------------- */
void oracle_decompose(const oracle_grid* grid, int32_t batch, const double* s, int32_t order,
                      int32_t refine_steps, double* resid, double* approx, double* theta,
                      double* coef, int64_t* index, double* energy, double* gap,
                      int32_t* flags) {
    int32_t n = grid->n;
    int64_t K = oracle_grid_size(grid);
    double step[4], lo[4], hi[4];
    oracle_refine_box(grid, step, lo, hi);
    double* p = (double*)malloc(sizeof(double) * (size_t)K);
    double* gs = (double*)malloc(sizeof(double) * (size_t)n);
    for (int32_t b = 0; b < batch; ++b) {
        double* r = resid + (size_t)b * n;
        double* a = approx ? approx + (size_t)b * n : NULL;
        memcpy(r, s + (size_t)b * n, sizeof(double) * (size_t)n);
        if (a) memset(a, 0, sizeof(double) * (size_t)n);
        int fl = 0;
        for (int32_t k = 0; k < n; ++k)
            if (!isfinite(r[k])) fl |= ORACLE_FLAG_NONFINITE;
        energy[(size_t)b * (order + 1)] = dot(r, r, n);
        for (int32_t k = 0; k < order; ++k) {
            size_t o = (size_t)b * order + k;
            oracle_correlate(grid, r, 0, K, p);
            double gp;
            int64_t best = oracle_argmax(p, K, &gp);
            double th0[4], th[4], J;
            oracle_grid_theta(grid, best, th0);
            if (refine_steps > 0)
                fl |= oracle_refine(grid->fs, n, r, th0, step, lo, hi, refine_steps, th, &J);
            else
                memcpy(th, th0, sizeof th);
            oracle_atom_unit(grid->fs, n, th, gs);
            double ck = dot(gs, r, n);
            for (int32_t t = 0; t < n; ++t) r[t] = r[t] - ck * gs[t];
            if (a)
                for (int32_t t = 0; t < n; ++t) a[t] = a[t] + ck * gs[t];
            memcpy(theta + 4 * o, th, sizeof th);
            coef[o] = ck;
            index[o] = best;
            gap[o] = gp;
            energy[(size_t)b * (order + 1) + k + 1] = dot(r, r, n);
        }
        flags[b] = fl & ~ORACLE_FLAG_LINESEARCH;
    }
    free(gs);
    free(p);
}

/* ---------------------------------------------------------------------------
 * The prior ACT that Sec. III-A contrasts with (Table "Comparison of
 * algorithmic properties"): atoms are not normalised to unit l2 norm (the
 * sampled real part of Eq. (1) keeps its analytic prefactor
 * (sqrt(pi) dt)^(-1/2)); the coarse search, the refinement and the
 * coefficient all use the original signal s rather than the residual; the
 * process repeats for each order, r_{k+1} = r_k - c g*, a_{k+1} = a_k + c g*.
 * ------------------------------------------------------------------------- */

/* (sqrt(pi) dt)^(-1/2) * real part of Eq. (1), sampled at t_k = k/fs. */
void oracle_atom_prior(double fs, int32_t n, const double theta[4], double* g) {
    oracle_atom_raw(fs, n, theta, g);
    double pref = 1.0 / sqrt(sqrt(ORACLE_PI) * exp(theta[3]));
    for (int32_t k = 0; k < n; ++k) g[k] = pref * g[k];
}

/* p_i = <g_i, s> with the prior ACT's (un-normalised) atoms. */
void oracle_correlate_prior(const oracle_grid* grid, const double* s, int64_t begin, int64_t count,
                            double* p) {
    int32_t n = grid->n;
#pragma omp parallel
    {
        double* g = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < count; ++j) {
            double th[4];
            oracle_grid_theta(grid, begin + j, th);
            oracle_atom_prior(grid->fs, n, th, g);
            p[j] = dot(g, s, n);
        }
        free(g);
    }
}

/* J(theta) = <s, g(theta)>^2 with the un-normalised atom, and its gradient:
 * with w = raw atom and P^2 = 1/(sqrt(pi) dt), J = P^2 <s,w>^2 and
 * dJ/dtheta_j = 2 P^2 <s,w> <s, d_j w>, plus -J for theta_3 = ln dt. */
double oracle_objective_prior(double fs, int32_t n, const double theta[4], const double* s,
                              double grad[4]) {
    double tc = theta[0], fc = theta[1], c = theta[2];
    double dt = exp(theta[3]);
    double p2 = 1.0 / (sqrt(ORACLE_PI) * dt);
    double sw = 0.0, sd[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - tc;
        double u = tau / dt;
        double e = exp(-0.5 * u * u);
        double ph = TWO_PI * (c * tau * tau + fc * tau);
        double co = cos(ph), si = sin(ph);
        double d[4];
        d[0] = e * ((tau / (dt * dt)) * co + TWO_PI * (2.0 * c * tau + fc) * si);
        d[1] = -TWO_PI * tau * e * si;
        d[2] = -TWO_PI * tau * tau * e * si;
        d[3] = (tau * tau / (dt * dt)) * e * co;
        sw += s[k] * e * co;
        for (int j = 0; j < 4; ++j) sd[j] += s[k] * d[j];
    }
    double J = p2 * sw * sw;
    if (grad) {
        for (int j = 0; j < 4; ++j) grad[j] = 2.0 * p2 * sw * sd[j];
        grad[3] -= J;
    }
    return J;
}

int oracle_refine_complex(double fs, int32_t n, const double* r, const double theta0[4], const double step[4],
                          const double lo[4], const double hi[4], int32_t steps, double theta_out[4], double* j_out) {
    return refine_core(fs, n, r, theta0, step, lo, hi, steps, theta_out, j_out, 2);
}

int oracle_refine_prior(double fs, int32_t n, const double* s, const double theta0[4],
                        const double step[4], const double lo[4], const double hi[4], int32_t steps,
                        double theta_out[4], double* j_out) {
    return refine_core(fs, n, s, theta0, step, lo, hi, steps, theta_out, j_out, 1);
}

/* The prior ACT over P orders (arguments as oracle_decompose; gap unused). */
void oracle_decompose_prior(const oracle_grid* grid, int32_t batch, const double* s, int32_t order,
                            int32_t refine_steps, double* resid, double* approx, double* theta,
                            double* coef, int64_t* index, double* energy, int32_t* flags) {
    int32_t n = grid->n;
    int64_t K = oracle_grid_size(grid);
    double step[4], lo[4], hi[4];
    oracle_refine_box(grid, step, lo, hi);
    double* p = (double*)malloc(sizeof(double) * (size_t)K);
    double* gs = (double*)malloc(sizeof(double) * (size_t)n);
    for (int32_t b = 0; b < batch; ++b) {
        const double* sb = s + (size_t)b * n;
        double* r = resid + (size_t)b * n;
        double* a = approx ? approx + (size_t)b * n : NULL;
        memcpy(r, sb, sizeof(double) * (size_t)n);
        if (a) memset(a, 0, sizeof(double) * (size_t)n);
        int fl = 0;
        for (int32_t k = 0; k < n; ++k)
            if (!isfinite(r[k])) fl |= ORACLE_FLAG_NONFINITE;
        energy[(size_t)b * (order + 1)] = dot(r, r, n);
        for (int32_t k = 0; k < order; ++k) {
            size_t o = (size_t)b * order + k;
            oracle_correlate_prior(grid, sb, 0, K, p);
            int64_t best = oracle_argmax(p, K, NULL);
            double th0[4], th[4], J;
            oracle_grid_theta(grid, best, th0);
            if (refine_steps > 0)
                fl |= oracle_refine_prior(grid->fs, n, sb, th0, step, lo, hi, refine_steps, th, &J);
            else
                memcpy(th, th0, sizeof th);
            oracle_atom_prior(grid->fs, n, th, gs);
            double ck = dot(gs, sb, n);
            for (int32_t t = 0; t < n; ++t) r[t] = r[t] - ck * gs[t];
            if (a)
                for (int32_t t = 0; t < n; ++t) a[t] = a[t] + ck * gs[t];
            memcpy(theta + 4 * o, th, sizeof th);
            coef[o] = ck;
            index[o] = best;
            energy[(size_t)b * (order + 1) + k + 1] = dot(r, r, n);
        }
        flags[b] = fl & ~ORACLE_FLAG_LINESEARCH;
    }
    free(gs);
    free(p);
}

/* ---------------------------------------------------------------------------
 * LEM-inspired hierarchical coarse-to-fine search (Sec. VII, Fig.
 * "Hierarchical LEM-inspired coarse-to-fine search"), per order on the
 * current residual:
 *   1. Latin-hypercube samples u (drawn by the caller, [samples][4] in [0,1))
 *      map to the parameter hull and snap to the coarsest step grid (level 0);
 *      each is projected (unit atom) onto the residual and the top-k distinct
 *      candidates by |<g, r>| are kept (ties: earlier candidate).
 *   2. For each refinement level l = 1..L, every kept candidate spawns the
 *      local family candidate + i * step_l, i_d in [-radius_d, radius_d]
 *      (members outside the hull dropped); all families are pooled and the
 *      top-k distinct are kept again.
 *   3. The best final candidate initialises the refinement (scales capped by
 *      the finest step), then c_k = <g*, r_k> and the residual update.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t samples, levels, topk, pad;
    int32_t radius[4];
    double step[8][4]; /* per level 0..levels, axes (t_c s, f_c Hz, c Hz/s, ln dt) */
} oracle_lem;

static double lem_snap(double x, double lo, double hi, double st) {
    if (!(hi > lo) || !(st > 0.0)) return lo;
    double v = lo + floor((x - lo) / st + 0.5) * st;
    if (v > hi) v = lo + floor((hi - lo) / st) * st;
    return v < lo ? lo : v;
}

/* top-k distinct candidates by |p| (ties: the earlier one); returns count */
static int lem_topk(const double* cand, const double* p, int m, int k, double* kept) {
    int nk = 0;
    char* used = (char*)calloc((size_t)(m > 0 ? m : 1), 1);
    while (nk < k) {
        int best = -1;
        for (int j = 0; j < m; ++j)
            if (!used[j] && (best < 0 || fabs(p[j]) > fabs(p[best]))) best = j;
        if (best < 0) break;
        used[best] = 1;
        int dup = 0;
        for (int a = 0; a < nk; ++a)
            if (kept[4 * a] == cand[4 * best] && kept[4 * a + 1] == cand[4 * best + 1] &&
                kept[4 * a + 2] == cand[4 * best + 2] && kept[4 * a + 3] == cand[4 * best + 3])
                dup = 1;
        if (dup) continue;
        memcpy(kept + 4 * nk, cand + 4 * best, 4 * sizeof(double));
        ++nk;
    }
    free(used);
    return nk;
}

static void lem_scores(double fs, int32_t n, const double* cand, int m, const double* r, double* p) {
#pragma omp parallel
    {
        double* g = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int j = 0; j < m; ++j) {
            oracle_atom_unit(fs, n, cand + 4 * j, g);
            p[j] = dot(g, r, n);
        }
        free(g);
    }
}

/* lhs: [batch][order][samples][4]; outputs as oracle_decompose (no index/gap). */
void oracle_lem_decompose(const oracle_grid* grid, const oracle_lem* cfg, int32_t batch, const double* s,
                          const double* lhs, int32_t order, int32_t refine_steps, double* resid,
                          double* approx, double* theta, double* coef, double* energy, int32_t* flags) {
    int32_t n = grid->n;
    double gstep[4], lo[4], hi[4];
    oracle_refine_box(grid, gstep, lo, hi);
    int fam = 1;
    for (int d = 0; d < 4; ++d) fam *= 2 * cfg->radius[d] + 1;
    int cap = cfg->samples > cfg->topk * fam ? cfg->samples : cfg->topk * fam;
    double* cand = (double*)malloc(sizeof(double) * 4 * (size_t)cap);
    double* p = (double*)malloc(sizeof(double) * (size_t)cap);
    double* kept = (double*)malloc(sizeof(double) * 4 * (size_t)cfg->topk);
    double* gs = (double*)malloc(sizeof(double) * (size_t)n);
    const double* fin = cfg->step[cfg->levels];
    for (int32_t b = 0; b < batch; ++b) {
        double* r = resid + (size_t)b * n;
        double* a = approx ? approx + (size_t)b * n : NULL;
        memcpy(r, s + (size_t)b * n, sizeof(double) * (size_t)n);
        if (a) memset(a, 0, sizeof(double) * (size_t)n);
        int fl = 0;
        for (int32_t k = 0; k < n; ++k)
            if (!isfinite(r[k])) fl |= ORACLE_FLAG_NONFINITE;
        energy[(size_t)b * (order + 1)] = dot(r, r, n);
        for (int32_t k = 0; k < order; ++k) {
            size_t o = (size_t)b * order + k;
            const double* u = lhs + (((size_t)b * order + k) * cfg->samples) * 4;
            for (int j = 0; j < cfg->samples; ++j)
                for (int d = 0; d < 4; ++d)
                    cand[4 * j + d] = lem_snap(lo[d] + u[4 * j + d] * (hi[d] - lo[d]), lo[d], hi[d], cfg->step[0][d]);
            lem_scores(grid->fs, n, cand, cfg->samples, r, p);
            int nk = lem_topk(cand, p, cfg->samples, cfg->topk, kept);
            for (int lv = 1; lv <= cfg->levels; ++lv) {
                const double* st = cfg->step[lv];
                int m = 0;
                for (int q = 0; q < nk; ++q)
                    for (int i0 = -cfg->radius[0]; i0 <= cfg->radius[0]; ++i0)
                        for (int i1 = -cfg->radius[1]; i1 <= cfg->radius[1]; ++i1)
                            for (int i2 = -cfg->radius[2]; i2 <= cfg->radius[2]; ++i2)
                                for (int i3 = -cfg->radius[3]; i3 <= cfg->radius[3]; ++i3) {
                                    const int ii[4] = {i0, i1, i2, i3};
                                    double th[4];
                                    int in = 1;
                                    for (int d = 0; d < 4; ++d) {
                                        th[d] = kept[4 * q + d] + (double)ii[d] * st[d];
                                        if (th[d] < lo[d] || th[d] > hi[d]) in = 0;
                                    }
                                    if (!in) continue;
                                    memcpy(cand + 4 * m, th, sizeof th);
                                    ++m;
                                }
                lem_scores(grid->fs, n, cand, m, r, p);
                nk = lem_topk(cand, p, m, cfg->topk, kept);
            }
            double th[4], J;
            if (refine_steps > 0)
                fl |= oracle_refine(grid->fs, n, r, kept, fin, lo, hi, refine_steps, th, &J);
            else
                memcpy(th, kept, sizeof th);
            oracle_atom_unit(grid->fs, n, th, gs);
            double ck = dot(gs, r, n);
            for (int32_t t = 0; t < n; ++t) r[t] = r[t] - ck * gs[t];
            if (a)
                for (int32_t t = 0; t < n; ++t) a[t] = a[t] + ck * gs[t];
            memcpy(theta + 4 * o, th, sizeof th);
            coef[o] = ck;
            energy[(size_t)b * (order + 1) + k + 1] = dot(r, r, n);
        }
        flags[b] = fl & ~ORACLE_FLAG_LINESEARCH;
    }
    free(gs);
    free(kept);
    free(p);
    free(cand);
}

/* ---------------------------------------------------------------------------
 * Complex (analytic) atoms, Eq. (1) literally: g = E e^{i phi}, phi =
 * 2 pi (c tau^2 + f_c tau), normalised over the samples present (|g|^2 = sum
 * E^2).  Selection and refinement use |<g_hat, r>|^2 = (a^2 + b^2) / sum E^2,
 * a = sum r E cos(phi), b = sum r E sin(phi).  A real signal is updated by its
 * orthogonal projection onto the real span of {Re g, Im g} (amplitude and
 * phase fitted by least squares), so the residual energy never increases.
 * ------------------------------------------------------------------------- */

/* |<g_hat, r>| for dictionary atoms [begin, begin+count). */
void oracle_correlate_complex(const oracle_grid* grid, const double* r, int64_t begin, int64_t count,
                              double* p) {
    int32_t n = grid->n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) {
        double th[4];
        oracle_grid_theta(grid, begin + j, th);
        double dt = exp(th[3]), a = 0.0, b = 0.0, q = 0.0;
        for (int32_t k = 0; k < n; ++k) {
            double tau = (double)k / grid->fs - th[0];
            double u = tau / dt;
            double e = exp(-0.5 * u * u);
            double ph = TWO_PI * (th[2] * tau * tau + th[1] * tau);
            a += r[k] * e * cos(ph);
            b += r[k] * e * sin(ph);
            q += e * e;
        }
        p[j] = q > 0.0 ? sqrt((a * a + b * b) / q) : 0.0;
    }
}

/* |<g_hat, r_t>| for m residuals at once (layout as oracle_correlate_many);
 * the sums run in the order of oracle_correlate_complex, so row t equals it
 * bit for bit. */
void oracle_correlate_complex_many(const oracle_grid* grid, int32_t m, const double* r, int64_t begin,
                                   int64_t count, double* p) {
    int32_t n = grid->n;
#pragma omp parallel
    {
        double* env = (double*)malloc(sizeof(double) * (size_t)n);
        double* co = (double*)malloc(sizeof(double) * (size_t)n);
        double* si = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < count; ++j) {
            double th[4];
            oracle_grid_theta(grid, begin + j, th);
            double dt = exp(th[3]), q = 0.0;
            for (int32_t k = 0; k < n; ++k) {
                double tau = (double)k / grid->fs - th[0];
                double u = tau / dt;
                double e = exp(-0.5 * u * u);
                double ph = TWO_PI * (th[2] * tau * tau + th[1] * tau);
                env[k] = e;
                co[k] = cos(ph);
                si[k] = sin(ph);
                q += e * e;
            }
            for (int32_t t = 0; t < m; ++t) {
                const double* rt = r + (size_t)t * n;
                double a = 0.0, b = 0.0;
                for (int32_t k = 0; k < n; ++k) {
                    a += rt[k] * env[k] * co[k];
                    b += rt[k] * env[k] * si[k];
                }
                p[(size_t)t * (size_t)count + (size_t)j] = q > 0.0 ? sqrt((a * a + b * b) / q) : 0.0;
            }
        }
        free(si);
        free(co);
        free(env);
    }
}

/* J = (a^2 + b^2) / q and its gradient in theta (SI units). */
double oracle_objective_complex(double fs, int32_t n, const double theta[4], const double* r, double grad[4]) {
    double tc = theta[0], fc = theta[1], c = theta[2];
    double dt = exp(theta[3]);
    double a = 0.0, b = 0.0, q = 0.0, da[4] = {0, 0, 0, 0}, db[4] = {0, 0, 0, 0}, dq[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - tc;
        double u = tau / dt;
        double e = exp(-0.5 * u * u);
        double ph = TWO_PI * (c * tau * tau + fc * tau);
        double co = cos(ph), si = sin(ph);
        /* dE/dtheta and dphi/dtheta */
        double de[4] = {e * tau / (dt * dt), 0.0, 0.0, e * tau * tau / (dt * dt)};
        double dp[4] = {-TWO_PI * (2.0 * c * tau + fc), TWO_PI * tau, TWO_PI * tau * tau, 0.0};
        a += r[k] * e * co;
        b += r[k] * e * si;
        q += e * e;
        for (int j = 0; j < 4; ++j) {
            da[j] += r[k] * (co * de[j] - e * si * dp[j]);
            db[j] += r[k] * (si * de[j] + e * co * dp[j]);
            dq[j] += 2.0 * e * de[j];
        }
    }
    if (!(q > 0.0)) {
        if (grad) grad[0] = grad[1] = grad[2] = grad[3] = 0.0;
        return 0.0;
    }
    double J = (a * a + b * b) / q;
    if (grad)
        for (int j = 0; j < 4; ++j) grad[j] = (2.0 * a * da[j] + 2.0 * b * db[j]) / q - J * dq[j] / q;
    return J;
}

/* Re and Im of the complex atom at theta (no normalisation). */
static void atom_complex(double fs, int32_t n, const double th[4], double* u, double* v) {
    double dt = exp(th[3]);
    for (int32_t k = 0; k < n; ++k) {
        double tau = (double)k / fs - th[0];
        double x = tau / dt;
        double e = exp(-0.5 * x * x);
        double ph = TWO_PI * (th[2] * tau * tau + th[1] * tau);
        u[k] = e * cos(ph);
        v[k] = e * sin(ph);
    }
}

/* least-squares amplitudes (alpha, beta) of r on {u, v}; 0 when singular */
static void fit2(const double* u, const double* v, const double* r, int32_t n, double* alpha, double* beta) {
    double uu = dot(u, u, n), vv = dot(v, v, n), uv = dot(u, v, n), ur = dot(u, r, n), vr = dot(v, r, n);
    double det = uu * vv - uv * uv;
    if (!(det > 1e-300 * (uu * vv > 0.0 ? uu * vv : 1.0)) || !(uu > 0.0)) {
        /* degenerate (e.g. f_c = c = 0 at t_c: v = 0): one-dimensional fit on u */
        *alpha = uu > 0.0 ? ur / uu : 0.0;
        *beta = 0.0;
        return;
    }
    *alpha = (vv * ur - uv * vr) / det;
    *beta = (uu * vr - uv * ur) / det;
}

int oracle_refine_complex(double fs, int32_t n, const double* r, const double theta0[4], const double step[4],
                          const double lo[4], const double hi[4], int32_t steps, double theta_out[4], double* j_out);

/* Re and Im of the raw complex atom, for callers. */
void oracle_atom_complex(double fs, int32_t n, const double theta[4], double* u, double* v) {
    atom_complex(fs, n, theta, u, v);
}

/* Amplitudes (ab[0], ab[1]) of the least-squares fit of r on the atom's parts. */
void oracle_fit_complex(double fs, int32_t n, const double theta[4], const double* r, double ab[2]) {
    double* u = (double*)malloc(sizeof(double) * (size_t)n);
    double* v = (double*)malloc(sizeof(double) * (size_t)n);
    atom_complex(fs, n, theta, u, v);
    fit2(u, v, r, n, &ab[0], &ab[1]);
    free(v);
    free(u);
}

/* Complex-atom MP; coef_re/coef_im [batch][order] are the amplitudes of Re g
 * and Im g of the raw atom; index/gap as oracle_decompose. */
void oracle_decompose_complex(const oracle_grid* grid, int32_t batch, const double* s, int32_t order,
                              int32_t refine_steps, double* resid, double* approx, double* theta,
                              double* coef_re, double* coef_im, int64_t* index, double* energy, double* gap,
                              int32_t* flags) {
    int32_t n = grid->n;
    int64_t K = oracle_grid_size(grid);
    double step[4], lo[4], hi[4];
    oracle_refine_box(grid, step, lo, hi);
    double* p = (double*)malloc(sizeof(double) * (size_t)K);
    double* u = (double*)malloc(sizeof(double) * (size_t)n);
    double* v = (double*)malloc(sizeof(double) * (size_t)n);
    for (int32_t b = 0; b < batch; ++b) {
        double* r = resid + (size_t)b * n;
        double* a = approx ? approx + (size_t)b * n : NULL;
        memcpy(r, s + (size_t)b * n, sizeof(double) * (size_t)n);
        if (a) memset(a, 0, sizeof(double) * (size_t)n);
        int fl = 0;
        for (int32_t k = 0; k < n; ++k)
            if (!isfinite(r[k])) fl |= ORACLE_FLAG_NONFINITE;
        energy[(size_t)b * (order + 1)] = dot(r, r, n);
        for (int32_t k = 0; k < order; ++k) {
            size_t o = (size_t)b * order + k;
            oracle_correlate_complex(grid, r, 0, K, p);
            double gp;
            int64_t best = oracle_argmax(p, K, &gp);
            double th0[4], th[4], J;
            oracle_grid_theta(grid, best, th0);
            if (refine_steps > 0)
                fl |= oracle_refine_complex(grid->fs, n, r, th0, step, lo, hi, refine_steps, th, &J);
            else
                memcpy(th, th0, sizeof th);
            atom_complex(grid->fs, n, th, u, v);
            double al, be;
            fit2(u, v, r, n, &al, &be);
            for (int32_t t = 0; t < n; ++t) {
                double w = al * u[t] + be * v[t];
                r[t] = r[t] - w;
                if (a) a[t] = a[t] + w;
            }
            memcpy(theta + 4 * o, th, sizeof th);
            coef_re[o] = al;
            coef_im[o] = be;
            index[o] = best;
            gap[o] = gp;
            energy[(size_t)b * (order + 1) + k + 1] = dot(r, r, n);
        }
        flags[b] = fl & ~ORACLE_FLAG_LINESEARCH;
    }
    free(v);
    free(u);
    free(p);
}

/* sum_k coef_k * unit_atom(theta_k) for one channel (Eq. (3)). */
void oracle_reconstruct(double fs, int32_t n, int32_t order, const double* theta,
                        const double* coef, double* out) {
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    memset(out, 0, sizeof(double) * (size_t)n);
    for (int32_t k = 0; k < order; ++k) {
        oracle_atom_unit(fs, n, theta + 4 * k, g);
        for (int32_t t = 0; t < n; ++t) out[t] = out[t] + coef[k] * g[t];
    }
    free(g);
}
