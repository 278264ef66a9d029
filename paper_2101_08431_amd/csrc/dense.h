// Dense linear algebra of the interior-point stage: Gauss-Newton Schur
// complement (eq. (20)), its tiled Cholesky factorisation and the triangular
// solves, on FP64 matrix cores.  Layouts are described in dense.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmfk {

// Components of Z_i = L_i^-1 Y stored per row: K rounded up to a multiple of
// 4 (the k-step of the matrix cores), zero-padded.
constexpr int zpad(int K) { return (K + 3) / 4 * 4; }

struct SchurArgs {
    const double *Z;        // [n][zpad(K)][ldY]: Z_i = L_i^-1 Y, zero for components >= K and columns >= m
    const double *XX;       // [n][K(K+1)/2]: X_ia X_ib, a >= b
    int64_t n, m, ldY;
    int npairs;             // 16 x 16 tile pairs (J >= L): T (T + 1) / 2, T = ceil(m / 16)
    int P;                  // row splits (P > 1: partial sums in `part`, then a reduction)
    int64_t rows_per_split;
    double *part;           // [P][npairs][K(K+1)/2][256]
    double *S;              // column-major, leading dimension ldS
    int64_t ldS;
    const double *GX;       // X^T X (K x K, device)
    const double *s, *Y;    // duals and factor of the columns, [K][ldY]
    double rho;
};

// Exact-Hessian Schur complement (eq. (27)): S = Q2bar - sum_i V_i^T V_i with
// V_i[p][(a, j)] = X_ia Z_i[p][j] + (L_i^-1)[p][a] R_ij, R = XY - M; V is
// written out row by row (k = i K + p) and the sum runs over k on matrix cores.
struct SchurExArgs {
    const double *Z;        // [n][zpad(K)][ldY]
    const double *X;        // [K][ldX]
    const double *Linv;     // [n][K][K]: (L_i^-1)[p][a] at (i*K + p)*K + a
    const double *R;        // [n][ldY]: R_ij = (XY - M)_ij, row-major
    int64_t n, m, ldX, ldY;
    int NT;                 // 64 x 64 tiles per side of the padded S
    double *S;
    int64_t ldS;
    const double *GX;
    const double *s, *Y;
    double rho;
};

// res = rhs - S v for the Gauss-Newton (eq. (20)) or exact-Hessian (eq. (27))
// Schur complement applied without forming S (FP64).
struct OpArgs {
    const double *Z;        // [n][zpad(K)][ldY]
    const double *X;        // [K][ldX]
    const double *Linv;     // [n][K][K] (exact Hessian)
    const double *R;        // [n][ldY]: (XY - M) rows (exact Hessian)
    int64_t n, m, ldX, ldY;
    const double *v;        // [Np], component-major (row a*m + j), zero past N = m K
    double *T;              // [n][ldY] work: t_i = Z_i^T V_i v
    double *H;              // [n][K] work: h_i = L_i^-T V_i v (exact Hessian)
    int S;                  // row splits of the column pass
    double *part;           // [S][K][ldY] work
    const double *GX, *s, *Y;
    double rho;
    const double *rhs;      // [Np]
    double *res;            // [Np] out
    int64_t Np;
};

struct CholArgs {
    double *S;              // column-major NT*64 x NT*64 (lower triangle used), leading dimension ldS
    int64_t ldS;
    int NT;                 // 64 x 64 tiles per side
    double *Dinv;           // [NT][64 x 64]: inverse of each diagonal factor tile, column-major
    int *fail;              // set to 1 on a non-positive pivot
};

struct SolveArgs {
    const double *S;
    int64_t ldS;
    int NT;
    const double *Dinv;
    const double *b;        // right-hand side (forward solve)
    double *y;              // solution (forward) / right-hand side overwritten by the solution (backward)
    unsigned *flags;        // [NT]
    unsigned epoch;
    int *fail;
};

int schur_chunks(int K);
hipError_t launch_xx(int K, const double *X, int64_t ldX, int64_t n, double *XX, hipStream_t st);
hipError_t launch_schur_gn(int K, const SchurArgs &g, hipStream_t st);
// The exact-Hessian Schur complement with V written out (k_vgen) in slabs of
// `slab` rows into V ([slab][ldV] doubles, or floats when f32; ldV >= NT*64, a
// multiple of 64) and summed by a matrix-core rank update per slab (k_syrk_v).
// Row splits per 128 x 128 tile of the exact-Hessian rank update for `tiles`
// tiles, within a partial-tile capacity of `cap` doubles (1: no split).
int syrk_splits(int64_t tiles, int64_t cap);
// kpart (capacity kpart_cap doubles, may be null): partial tiles when the rows
// of each slab are split over several blocks per tile, which the launcher does
// when the 128 x 128 tiles are too few to fill the chip evenly.
hipError_t launch_schur_exact_rows(int K, const SchurExArgs &g, void *V, int64_t ldV, int64_t slab, bool f32,
                                   double *kpart, int64_t kpart_cap, hipStream_t st);
hipError_t launch_schur_apply(int K, bool exact, const OpArgs &g, hipStream_t st);
hipError_t launch_axpy(double *y, const double *x, int64_t count, hipStream_t st);
// Linv[i][p][a] = (L_i^-1)[p][a] from the packed factors Lq ([K(K+1)/2 + K][ldX]:
// lower triangle row by row, then the reciprocal diagonal).
hipError_t launch_linv(int K, const double *Lq, int64_t ldX, int64_t n, double *Linv, hipStream_t st);
// R[i*ldY + j] = (X Y - M)_ij for j < m, 0 for m <= j < ldY (M column-major, ldM).
hipError_t launch_residual_rows(int K, const double *M, int64_t ldM, const double *X, int64_t ldX,
                                const double *Y, int64_t ldY, int64_t n, int64_t m, double *R, hipStream_t st);
hipError_t launch_pad_identity(double *S, int64_t ldS, int64_t N, int64_t Np, hipStream_t st);
hipError_t launch_cholesky(const CholArgs &g, hipStream_t st);
hipError_t launch_solve(const SolveArgs &fwd, const SolveArgs &bwd, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t st);

}  // namespace nmfk
