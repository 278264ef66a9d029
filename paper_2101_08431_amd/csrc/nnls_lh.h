// Warm-started Lawson-Hanson NNLS in Gram form, one problem per lane.
//
// Solves min 1/2 x^T G x - b^T x subject to x >= 0 (eq. (2) of Sec. II with
// G = C^T C and b = C^T d), starting from the previous solution of the same
// row or column and its passive set, as the warm-start strategy of Sec. II
// prescribes.  The minimiser is unique for G of full rank, so the result does
// not depend on the starting point.
//
// The linear solves z_P = G_PP^-1 b_P use a Cholesky factorisation of the
// full K x K matrix in which the rows and columns outside P are replaced by
// those of the identity and b by 0 outside P.  That factor restricted to P is
// the Cholesky factor of G_PP (the extra terms are exact zeros), and z is 0
// off P.  Every index is a compile-time constant, so the factor, x, z and the
// dual vector live in registers; G is read from LDS (one copy per block).
//
// Rules where the cited method leaves a choice (the same rules as the CPU
// oracle, written independently):
//   optimality when w_a <= tol for every a outside P, w = b - G x,
//     tol = 10 K eps max_a (|b_a| + sum_c |G_ac| x_c);
//   the entering index is the first of largest w;
//   the blocking index is the first of smallest ratio x_a / (x_a - z_a); it is
//     set to exactly 0 and every passive index with x_a <= 0 leaves P;
//   an index with G_aa <= 1e-14 max G is never entered;
//   an index whose first solve after entering is <= 0, or whose entry breaks the
//     factorisation, leaves P and is not tried again in this solve;
//   at most 6K + 10 solves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmfk {

template <int K>
__device__ __forceinline__ double sel(const double (&v)[K], int idx) {
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a)
        if (a == idx) r = v[a];
    return r;
}

template <int K>
__device__ __forceinline__ void put(double (&v)[K], int idx, double val) {
#pragma unroll
    for (int a = 0; a < K; ++a)
        if (a == idx) v[a] = val;
}

// 1/sqrt(v) for a normal v > 0: the hardware estimate (v_rsq_f64) refined by
// two Newton steps y <- y + (y/2)(1 - v y^2), each of which squares the
// relative error, so the result is within a few ulp.  Its dependent chain is
// about a third of a correctly rounded sqrt followed by a division.
__device__ __forceinline__ double rsqrt_newton(double v) {
    double y = __builtin_amdgcn_rsq(v);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-v * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// z = (G masked to P)^-1 (b masked to P).  Returns false if a pivot on P is
// not positive.  The factor keeps only the reciprocals of its diagonal (the
// solves multiply by them), taken as reciprocal square roots of the pivots.
template <int K>
__device__ __forceinline__ bool masked_solve(const double *G, const double (&b)[K], uint32_t P,
                                             double (&z)[K]) {
    double L[K * (K + 1) / 2];   // off-diagonal entries only are read
    double inv[K];
    bool ok = true;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const bool pr = (P >> r) & 1u;
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            const bool pc = (P >> c) & 1u;
            double v = (pr && pc) ? G[r * K + c] : (r == c ? 1.0 : 0.0);
#pragma unroll
            for (int q = 0; q < c; ++q) v -= L[r * (r + 1) / 2 + q] * L[c * (c + 1) / 2 + q];
            if (r == c) {
                ok = ok && (v > 0.0);
                inv[r] = rsqrt_newton(v > 0.0 ? v : 1.0);
            } else {
                L[r * (r + 1) / 2 + c] = v * inv[c];
            }
        }
    }
    double t[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        double v = ((P >> r) & 1u) ? b[r] : 0.0;
#pragma unroll
        for (int q = 0; q < r; ++q) v -= L[r * (r + 1) / 2 + q] * t[q];
        t[r] = v * inv[r];
    }
#pragma unroll
    for (int r = K - 1; r >= 0; --r) {
        double v = t[r];
#pragma unroll
        for (int q = r + 1; q < K; ++q) v -= L[q * (q + 1) / 2 + r] * z[q];
        z[r] = v * inv[r];
    }
    return ok;
}

struct LhResult {
    uint32_t P;
    int solves;
    int status;   // 0 ok, -2 solve cap, -3 breakdown after a blocking step
};

// x: in = previous solution (>= 0), out = new solution.  gmax = max_a G_aa.
template <int K>
__device__ LhResult lh_warm(const double *G, double gmax, const double (&b)[K], double (&x)[K]) {
    uint32_t barred = 0, P = 0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        if (!(G[a * K + a] > 1e-14 * gmax)) barred |= 1u << a;
        if (x[a] > 0.0 && !((barred >> a) & 1u))
            P |= 1u << a;
        else
            x[a] = 0.0;
    }
    const int cap = 6 * K + 10;
    int solves = 0, status = 0, entered = -1;
    bool need_solve = (P != 0u), done = false;
    double z[K];
    while (!done) {
        if (need_solve) {
            bool first = true;
            while (true) {
                if (++solves > cap) { status = -2; done = true; break; }
                const bool ok = masked_solve<K>(G, b, P, z);
                if (!ok) {
                    if (entered >= 0 && first) {
                        P &= ~(1u << entered);
                        barred |= 1u << entered;
                        put<K>(x, entered, 0.0);
                    } else if (entered < 0) {
                        // the warm-start set is numerically singular: start cold
                        P = 0u;
#pragma unroll
                        for (int a = 0; a < K; ++a) x[a] = 0.0;
                    } else {
                        status = -3;
                        done = true;
                    }
                    break;
                }
                bool feas = true;
#pragma unroll
                for (int a = 0; a < K; ++a)
                    if (((P >> a) & 1u) && !(z[a] > 0.0)) feas = false;
                if (feas) {
#pragma unroll
                    for (int a = 0; a < K; ++a) x[a] = ((P >> a) & 1u) ? z[a] : 0.0;
                    break;
                }
                if (first && entered >= 0 && !(sel<K>(z, entered) > 0.0)) {
                    P &= ~(1u << entered);
                    barred |= 1u << entered;
                    put<K>(x, entered, 0.0);
                    break;
                }
                first = false;
                double alpha = 0.0;
                int q = -1;
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    if (((P >> a) & 1u) && !(z[a] > 0.0)) {
                        const double ra = x[a] / (x[a] - z[a]);
                        if (q < 0 || ra < alpha) { alpha = ra; q = a; }
                    }
                }
#pragma unroll
                for (int a = 0; a < K; ++a)
                    if ((P >> a) & 1u) x[a] += alpha * (z[a] - x[a]);
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    if (a == q) x[a] = 0.0;
                    if (((P >> a) & 1u) && !(x[a] > 0.0)) { x[a] = 0.0; P &= ~(1u << a); }
                }
            }
            if (done) break;
        }
        // optimality test on the dual vector
        double tol = 0.0, wj = 0.0;
        int j = -1;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double v = b[a], s = fabs(b[a]);
#pragma unroll
            for (int c = 0; c < K; ++c) {
                v -= G[a * K + c] * x[c];
                s += fabs(G[a * K + c]) * x[c];
            }
            tol = s > tol ? s : tol;
            if (!(((P | barred) >> a) & 1u)) {
                if (j < 0 || v > wj) { j = a; wj = v; }
            }
        }
        tol *= 10.0 * K * 2.220446049250313e-16;
        if (j < 0 || !(wj > tol)) break;
        P |= 1u << j;
        entered = j;
        need_solve = true;
    }
    LhResult r;
    r.P = P;
    r.solves = solves;
    r.status = status;
    return r;
}

}  // namespace nmfk
