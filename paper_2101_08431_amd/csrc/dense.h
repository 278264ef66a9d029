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
hipError_t launch_pad_identity(double *S, int64_t ldS, int64_t N, int64_t Np, hipStream_t st);
hipError_t launch_cholesky(const CholArgs &g, hipStream_t st);
hipError_t launch_solve(const SolveArgs &fwd, const SolveArgs &bwd, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t st);

}  // namespace nmfk
