/*
 * FP64 CPU oracle for the ANLS stage of the two-stage NMF of Gu, Du and
 * Billinge, "A fast two-stage algorithm for non-negative matrix factorization
 * in streaming data" (Sec. II and Alg. 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or loads this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code with the GPU library.
 *
 * What it computes.  Alg. 1 alternates two convex subproblems, X first, then Y.
 * Each splits into independent single right-hand-side non-negative least
 * squares problems, eq. (2): min 1/2 ||C x - d||^2, x >= 0, with C = Y^T and d a
 * row of M (the X-half), or C = X and d a column of M (the Y-half).  With
 * G = C^T C and b = C^T d the problem is min 1/2 x^T G x - b^T x, x >= 0; for a
 * G of full rank it is strictly convex, so its minimiser is unique and any exact
 * method returns it.  The oracle uses the active-set method of Lawson and
 * Hanson that Sec. II names, in its plain cold-started form (every problem
 * starts from x = 0): the result does not depend on warm starts, so the
 * paper's warm-start strategy is left to the fast path.
 *
 * Stage-1 stop rule (Sec. IV): ||(x_t, y_t) - (x_{t+1}, y_{t+1})||
 * <= eps_STOL (1 + ||(x_t, y_t)||), Euclidean norm over all entries.
 *
 * Layouts follow the vec conventions under eq. (3): x = vec(X^T) and
 * y = vec(Y), so
 *   X   n x k row-major, row i at X[i*k]
 *   Yt  m x k row-major, column j of Y at Yt[j*k]
 *   M   column-major, element (i, j) at M[j*ldm + i]
 *
 * Readings where the paper is silent (the Lawson-Hanson method is cited, not
 * printed):
 *   - optimality test on the dual vector w = b - G x: stop when every index
 *     outside the passive set has w_a <= tol, with
 *     tol = 10 k eps max_a (|b_a| + sum_c |G_ac| x_c), eps = 2^-52;
 *   - the entering index is the first index of largest w;
 *   - the blocking step takes the first index of smallest ratio, sets it to
 *     exactly 0, and drops every passive index whose value is <= 0;
 *   - an index with G_aa <= 1e-14 max_c G_cc never enters (a zero column of C);
 *   - an index whose first solve after entering is <= 0, or whose entry breaks
 *     the Cholesky factorisation, is dropped and not tried again in this solve;
 *   - at most 6k + 10 linear solves per problem (never reached on SPD input).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KMAX 32

int orc_kmax(void) { return ORC_KMAX; }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* z_P = G_PP^{-1} b_P by a Cholesky factorisation of the principal submatrix
 * G_PP, z = 0 outside P.  Returns 0, or -1 if a pivot is not positive. */
static int solve_passive(int k, const double *G, const double *b, uint32_t P, double *z) {
    int idx[ORC_KMAX];
    double L[ORC_KMAX * ORC_KMAX];
    double t[ORC_KMAX];
    int p = 0;
    for (int a = 0; a < k; ++a) {
        z[a] = 0.0;
        if (P & (1u << a)) idx[p++] = a;
    }
    for (int r = 0; r < p; ++r) {
        for (int c = 0; c <= r; ++c) {
            double v = G[idx[r] * k + idx[c]];
            for (int q = 0; q < c; ++q) v -= L[r * p + q] * L[c * p + q];
            if (r == c) {
                if (!(v > 0.0)) return -1;
                L[r * p + r] = sqrt(v);
            } else {
                L[r * p + c] = v / L[c * p + c];
            }
        }
    }
    for (int r = 0; r < p; ++r) { /* L t = b_P */
        double v = b[idx[r]];
        for (int q = 0; q < r; ++q) v -= L[r * p + q] * t[q];
        t[r] = v / L[r * p + r];
    }
    for (int r = p - 1; r >= 0; --r) { /* L^T z_P = t */
        double v = t[r];
        for (int q = r + 1; q < p; ++q) v -= L[q * p + r] * z[idx[q]];
        z[idx[r]] = v / L[r * p + r];
    }
    return 0;
}

/* Lawson-Hanson NNLS in Gram form, cold start.  G is k x k row-major.
 * On return x >= 0 holds the minimiser and *passive the set {a : x_a > 0} as a
 * bit mask.  Returns 0 on success, -2 if the solve cap was hit (x is then the
 * last feasible iterate).  *nsolve, if given, receives the number of linear
 * solves. */
int orc_nnls(int k, const double *G, const double *b, double *x, uint32_t *passive, int *nsolve) {
    double w[ORC_KMAX], z[ORC_KMAX];
    uint32_t P = 0, barred = 0;
    int solves = 0, status = 0;
    const int cap = 6 * k + 10;
    double gmax = 0.0;
    for (int a = 0; a < k; ++a) {
        x[a] = 0.0;
        if (G[a * k + a] > gmax) gmax = G[a * k + a];
    }
    for (int a = 0; a < k; ++a)
        if (!(G[a * k + a] > 1e-14 * gmax)) barred |= 1u << a;

    for (;;) {
        /* dual vector and optimality test */
        double tol = 0.0;
        for (int a = 0; a < k; ++a) {
            double v = b[a], s = fabs(b[a]);
            for (int c = 0; c < k; ++c) {
                v -= G[a * k + c] * x[c];
                s += fabs(G[a * k + c]) * x[c];
            }
            w[a] = v;
            if (s > tol) tol = s;
        }
        tol *= 10.0 * k * 2.220446049250313e-16;
        int j = -1;
        for (int a = 0; a < k; ++a) {
            if ((P | barred) & (1u << a)) continue;
            if (j < 0 || w[a] > w[j]) j = a;
        }
        if (j < 0 || !(w[j] > tol)) break;
        P |= 1u << j;

        /* inner loop: solve on P, step back to feasibility while needed */
        int first = 1;
        for (;;) {
            if (++solves > cap) { status = -2; goto done; }
            if (solve_passive(k, G, b, P, z) != 0) {
                /* the entering index made G_PP numerically singular */
                P &= ~(1u << j);
                barred |= 1u << j;
                x[j] = 0.0;
                if (!first) { status = -3; goto done; }
                break;
            }
            int feasible = 1;
            for (int a = 0; a < k; ++a)
                if ((P & (1u << a)) && !(z[a] > 0.0)) feasible = 0;
            if (feasible) {
                for (int a = 0; a < k; ++a) x[a] = (P & (1u << a)) ? z[a] : 0.0;
                break;
            }
            if (first && !(z[j] > 0.0)) {
                /* rounding made the entering index non-positive */
                P &= ~(1u << j);
                barred |= 1u << j;
                x[j] = 0.0;
                break;
            }
            first = 0;
            double alpha = 0.0;
            int q = -1;
            for (int a = 0; a < k; ++a) {
                if (!(P & (1u << a)) || z[a] > 0.0) continue;
                double ra = x[a] / (x[a] - z[a]);
                if (q < 0 || ra < alpha) { alpha = ra; q = a; }
            }
            for (int a = 0; a < k; ++a)
                if (P & (1u << a)) x[a] += alpha * (z[a] - x[a]);
            x[q] = 0.0;
            for (int a = 0; a < k; ++a)
                if ((P & (1u << a)) && !(x[a] > 0.0)) { x[a] = 0.0; P &= ~(1u << a); }
        }
    }
done:
    if (passive) *passive = P;
    if (nsolve) *nsolve = solves;
    return status;
}

/* X-half of Alg. 1: every row i of X solves eq. (2) with C = Y^T, d = row i of
 * M, i.e. G = Y Y^T and b = (M Y^T)_i.  masks (may be NULL) receives the
 * passive set of each row.  Returns the number of rows whose solve failed. */
int orc_half_x(int64_t n, int64_t m, int k, const double *M, int64_t ldm,
               double *X, const double *Yt, uint32_t *masks) {
    double G[ORC_KMAX * ORC_KMAX];
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
            double v = 0.0;
            for (int64_t j = 0; j < m; ++j) v += Yt[j * k + a] * Yt[j * k + c];
            G[a * k + c] = v;
        }
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t i = 0; i < n; ++i) {
        double b[ORC_KMAX];
        uint32_t P;
        for (int a = 0; a < k; ++a) {
            double v = 0.0;
            for (int64_t j = 0; j < m; ++j) v += M[j * ldm + i] * Yt[j * k + a];
            b[a] = v;
        }
        if (orc_nnls(k, G, b, X + i * k, &P, NULL) != 0) bad += 1;
        if (masks) masks[i] = P;
    }
    return bad;
}

/* Y-half of Alg. 1: every column j of Y solves eq. (2) with C = X, d = column j
 * of M, i.e. G = X^T X and b = (X^T M)_j. */
int orc_half_y(int64_t n, int64_t m, int k, const double *M, int64_t ldm,
               const double *X, double *Yt, uint32_t *masks) {
    double G[ORC_KMAX * ORC_KMAX];
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
            double v = 0.0;
            for (int64_t i = 0; i < n; ++i) v += X[i * k + a] * X[i * k + c];
            G[a * k + c] = v;
        }
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t j = 0; j < m; ++j) {
        double b[ORC_KMAX];
        uint32_t P;
        for (int a = 0; a < k; ++a) {
            double v = 0.0;
            for (int64_t i = 0; i < n; ++i) v += X[i * k + a] * M[j * ldm + i];
            b[a] = v;
        }
        if (orc_nnls(k, G, b, Yt + j * k, &P, NULL) != 0) bad += 1;
        if (masks) masks[j] = P;
    }
    return bad;
}

/* 1/2 ||X Y - M||_F^2 from the residual itself, eq. (1). */
double orc_objective(int64_t n, int64_t m, int k, const double *M, int64_t ldm,
                     const double *X, const double *Yt) {
    double f = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : f)
    for (int64_t j = 0; j < m; ++j) {
        double fj = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double v = -M[j * ldm + i];
            for (int a = 0; a < k; ++a) v += X[i * k + a] * Yt[j * k + a];
            fj += v * v;
        }
        f += fj;
    }
    return 0.5 * f;
}

/* Alg. 1 from the given (X, Yt), in place, for at most max_sweeps sweeps.
 * A sweep is the X-half followed by the Y-half.  With eps_stol >= 0 it stops
 * after the first sweep that meets the Sec. IV step rule; with eps_stol < 0 it
 * runs exactly max_sweeps sweeps.  stats (may be NULL) receives
 * {sweeps done, stop rule met (0/1), last step norm, last ||(x_t, y_t)||,
 *  failed NNLS solves}.  Returns the number of sweeps done. */
int orc_anls(int64_t n, int64_t m, int k, const double *M, int64_t ldm,
             double *X, double *Yt, double eps_stol, int max_sweeps,
             uint32_t *xmask, uint32_t *ymask, double *stats) {
    double *Xo = (double *)malloc(sizeof(double) * (size_t)(n * k));
    double *Yo = (double *)malloc(sizeof(double) * (size_t)(m * k));
    int sweeps = 0, met = 0, bad = 0;
    double step = 0.0, nrm = 0.0;
    if (!Xo || !Yo) { free(Xo); free(Yo); return -1; }
    while (sweeps < max_sweeps) {
        memcpy(Xo, X, sizeof(double) * (size_t)(n * k));
        memcpy(Yo, Yt, sizeof(double) * (size_t)(m * k));
        bad += orc_half_x(n, m, k, M, ldm, X, Yt, xmask);
        bad += orc_half_y(n, m, k, M, ldm, X, Yt, ymask);
        ++sweeps;
        double d2 = 0.0, n2 = 0.0;
        for (int64_t q = 0; q < n * k; ++q) {
            double d = X[q] - Xo[q];
            d2 += d * d;
            n2 += Xo[q] * Xo[q];
        }
        for (int64_t q = 0; q < m * k; ++q) {
            double d = Yt[q] - Yo[q];
            d2 += d * d;
            n2 += Yo[q] * Yo[q];
        }
        step = sqrt(d2);
        nrm = sqrt(n2);
        if (eps_stol >= 0.0 && step <= eps_stol * (1.0 + nrm)) { met = 1; break; }
    }
    if (stats) {
        stats[0] = sweeps;
        stats[1] = met;
        stats[2] = step;
        stats[3] = nrm;
        stats[4] = bad;
    }
    free(Xo);
    free(Yo);
    return sweeps;
}
