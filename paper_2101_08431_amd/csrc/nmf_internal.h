// Internal declarations shared by the HIP sources of the NMF library.
// Device layouts (all double unless noted):
//   M      [m_cap][ldM]   column j (one time instant) contiguous
//   X      [K][ldX]       component-major: X[a*ldX + i] = X_ia
//   Y      [K][ldY]       Y[a*ldY + j] = Y_aj
//   xmask  [ldX] u32, ymask [ldY] u32: passive set of each row / column
// Component-major factors make every per-row (per-column) access of a wave
// a contiguous 512-byte load or store.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmfk {

constexpr int KMAX = 16;
constexpr int NTHR = 256;      // threads per block (4 waves of 64)
constexpr int XTILE = 64;      // rows of X per X-half tile (one row per lane)
constexpr int YVALS = 64;      // J*K partial sums per Y-half tile, padded to a wave
constexpr int NST = 8;         // doubles per tile statistics record
constexpr int XCHUNK = 256;    // columns of Y staged in LDS at a time

// Tile statistics record (per X-half or Y-half tile)
enum { ST_STEP2 = 0, ST_NORM2 = 1, ST_EG2 = 2, ST_EC2 = 3, ST_SOLVES = 4, ST_FAILS = 5,
       ST_CHANGES = 6, ST_SPARE = 7 };

struct DevStatus {
    double step2, norm2;          // last sweep: ||delta (x, y)||^2 and ||(x_t, y_t)||^2
    double ex_g2, ex_c2;          // X part of E(.;0) at the iterate before the last sweep
    double ey_g2, ey_c2;          // Y part of E(.;0) at the current iterate
    double ey_g2_prev, ey_c2_prev;
    double E_prev;                // E(.;0) at the iterate before the last sweep (-1: unknown)
    double E_cur;                 // E(.;0) at the current iterate from a measure pass (-1: unknown)
    double solves, fails, changes;
    double eps_stol;
    long long sweeps;
    int converged;
    int max_sweeps;
    double f_direct;              // 1/2 ||XY - M||^2 from the last direct pass
};

// Parameters of the stage-1 kernels.
struct AnlsParams {
    int64_t n, m, ldM, ldX, ldY;
    const double *M;
    double *X, *Y;
    uint32_t *xmask, *ymask;
    double *bx_part;   // [Sx][K][ldX]
    double *by_part;   // [Tm][Sy][YVALS]
    double *gx_part;   // [Tn][K*K]
    double *gy_part;   // [Tm][K*K]
    double *xstat;     // [Tn][NST]
    double *ystat;     // [Tm][NST]
    unsigned *cnt_x;   // [Tn]
    unsigned *cnt_y;   // [Tm]
    unsigned *cnt_fin; // [4]
    DevStatus *st;
    int Sx, Tn, xcols;
    int Sy, Tm, yrows;
    int mode;          // X-half: 0 = solve, 1 = measure E only; Y-half: 0 = sweep, 2 = appended columns
};

// Launchers (anls.hip).  All enqueue on `s` and return hipSuccess or an error.
hipError_t launch_xhalf(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_yhalf(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_measure_finish(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_gram_y_init(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_objective(int K, const AnlsParams &p, double *part, int nblk, hipStream_t s);
hipError_t launch_check_finite(const double *M, int64_t n, int64_t m, int64_t ldM, double *part,
                               int nblk, hipStream_t s);
hipError_t launch_factor_in(int K, const double *src_x, const double *src_y, const AnlsParams &p,
                            unsigned *bad, hipStream_t s);
hipError_t launch_factor_out(int K, const AnlsParams &p, double *dst_x, double *dst_y, hipStream_t s);
hipError_t launch_copy_columns_warm(int K, const AnlsParams &p, int64_t j_from, int64_t j0,
                                    int64_t j1, hipStream_t s);

int yhalf_cols(int K);   // columns per Y-half tile, J = YVALS / K

}  // namespace nmfk
