// Stage 2 of the two-stage NMF (Sec. III, IV, Alg. 3): transition and the
// primal-dual line-search interior-point iterations, on the device, with the
// host steering the loop tests from a few device-computed scalars.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/nmf.h"
#include "nmf_internal.h"

namespace nmfk {

constexpr int PARTW = 16;      // doubles per block record of the small reductions
constexpr int NTRIAL = 16;     // Armijo trial steps evaluated per batch

// Small device-resident results (k x k matrices and reduction outputs).
struct IpmScal {
    double GX[KMAX * KMAX];    // X^T X at the current point
    double GY[KMAX * KMAX];    // Y Y^T at the current point
    double XtV[KMAX * KMAX];   // X^T V, V_i = Q1bar_i^-1 b1_i
    double T[KMAX * KMAX];     // dY Y^T
    unsigned fin_cnt, fin_pad; // arrivals of the blocks of a kernel that reduces its own records
    double out[4 * PARTW];     // outputs of the last k_finish calls
    double f;                  // 1/2 ||XY - M||^2 at the current point
    int chol_fail;
    int solve_fail;            // 2: a triangular-solve block timed out waiting for its predecessor
};

struct IpmState {
    bool bound = false;
    int64_t n = 0, m_cap = 0, ldX = 0, ldY = 0, ldS = 0;
    int K = 0;
    // device buffers (component-major [K][ld] unless noted)
    double *r = nullptr, *s = nullptr;         // duals
    double *dx = nullptr, *dy = nullptr, *dr = nullptr, *ds = nullptr;
    double *gx = nullptr, *gy = nullptr;       // graX, graY
    double *V = nullptr;                       // Q1bar_i^-1 b1_i per row
    double *tX = nullptr, *tY = nullptr;       // residual products (exact Hessian)
    double *Lq = nullptr;                      // [K(K+1)/2 + K][ldX]: Cholesky of Q1bar_i and 1/diag
    double *Linv = nullptr;                    // [n][K][K]: L_i^-1 (exact Hessian)
    double *Rrow = nullptr;                    // [n][ldY]: residual XY - M, row-major (exact Hessian)
    double *Z = nullptr;                       // [n][K][ldY]: L_i^-1 Y
    double *S = nullptr;                       // [ldS][ldS] column-major, lower triangle used
    double *vec = nullptr, *vec2 = nullptr;    // [ldS] right-hand side / solution
    double *XX = nullptr;                      // [n][K(K+1)/2] products X_ia X_ib
    double *Dinv = nullptr;                    // [ldS/64][64*64] inverses of the diagonal factor tiles
    double *spart = nullptr;                   // Schur row-split partial sums (P > 1)
    // mixed precision (nmf_set_ipm_precision): exact-Hessian Schur formation in
    // FP32, the direction refined against the FP64 operator
    int mixed = 0, refine = 2;
    double *rhs0 = nullptr, *dacc = nullptr;   // [ldS] right-hand side, accumulated direction
    double *Top = nullptr, *Hop = nullptr;     // [n][ldY], [n][K] operator work
    double *opart = nullptr;                   // [OPS][K][ldY] operator partials
    double *Vex = nullptr;                     // [vrows][ldS] rows of the exact-Hessian factor V
    int64_t vrows = 0;
    IpmScal *hsc = nullptr;                    // pinned host copy of the scalar block (owner: the context)
    double *kpart = nullptr;                   // partial tiles of the split exact-Hessian rank update
    int64_t kpart_cap = 0;                     // its capacity in doubles
    unsigned *flags = nullptr;                 // [3][ldS/64] hand-over flags: factor, forward, backward solve
    unsigned epoch = 0;                        // last flag value used
    bool flags_ready = false;
    int P = 1;                                 // row splits of the Schur formation
    double *part = nullptr;                    // [nblk][PARTW] block records
    double *fpart = nullptr;                   // [Tn * Sx] objective partials
    IpmScal *sc = nullptr;
    // host-side state of Alg. 3
    double mu = 0, rho = 0, eps_mu = 0, E0 = 0, Emu = 0, sigma = 0, f = 0, slope = 0;
    double S1 = 0, C0 = 0, Cmu = 0, SR = 0;    // KKT sums at the current point
    int flag = 0, at_mu = 0;
    bool in_inner = false;                     // inside the inner loop of the current mu
    bool S_gn_valid = false;                   // S holds the factored Gauss-Newton Schur matrix of this point
    int64_t iters = 0, outer = 0, backtracks = 0, exact_steps = 0, fallbacks = 0, cap_hits = 0;
    // optional device timing of the dense steps (nmf_ipm_profile): events
    // around each Gauss-Newton / exact Schur formation, each factorisation
    // and each pair of triangular solves; prof_ms / prof_n accumulate
    bool prof = false;
    hipEvent_t pev[2] = {nullptr, nullptr};
    double prof_ms[4] = {0, 0, 0, 0};          // GN formation, exact formation, Cholesky, solve pair
    int64_t prof_n[4] = {0, 0, 0, 0};
    std::string err;
};

size_t ipm_workspace_bytes(int64_t n, int64_t m_cap, int K);
nmf_status ipm_bind(IpmState &s, uint8_t *base, int64_t n, int64_t m_cap, int K);
nmf_status ipm_transition(IpmState &s, const AnlsParams &p, const nmf_options &o, hipStream_t st);
nmf_status ipm_iterate(IpmState &s, const AnlsParams &p, const nmf_options &o, int iters, hipStream_t st);
nmf_status ipm_report(IpmState &s, nmf_report *r, double ms1, double ms2);
nmf_status ipm_export(IpmState &s, const AnlsParams &p, hipStream_t st);
nmf_status ipm_get_duals(IpmState &s, const AnlsParams &p, double *R, double *S, hipStream_t st);
const char *ipm_last_error(const IpmState &s);

}  // namespace nmfk
