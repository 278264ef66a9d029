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
constexpr int NTHR = 256;      // threads of the element-wise and reduction kernels
constexpr int WTHR = 64;       // one wave
// Threads of the stage-1 NNLS kernels (one problem per lane): one wave up to
// k = 8; beyond, four waves, so that the k^2-entry Gram records of the other
// half are summed by enough threads.  Records are written per wave either way.
constexpr int nnls_threads(int K) { return K <= 8 ? 64 : 256; }
constexpr int SWAVES = 8;      // waves of the streaming kernels
constexpr int STHR = 64 * SWAVES;
constexpr int XTILE = 64;      // rows of M per X-stream tile (one row per lane)
constexpr int YVALS = 64;      // J*K partial sums per Y-stream column tile, padded to a wave
constexpr int NST = 8;         // doubles per block statistics record
constexpr int XCHUNK = 256;    // columns of Y staged in LDS at a time

// Block statistics record of the NNLS kernels
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
    int pad_;
    long long max_sweeps;         // the stop rule also holds once sweeps reaches this count
    double f_direct;              // 1/2 ||XY - M||^2 from the last direct pass
};

// Parameters of the stage-1 kernels.  One sweep = k_xstream, k_xnnls,
// k_ystream, k_ynnls; every hand-over between blocks crosses a kernel
// boundary except the sweep summary at the end of k_ynnls.  A half may run as
// one kernel instead (k_xfused, k_yfused; fx, fy): each tile's splits stream
// as before and the last of them to finish solves the tile.
struct AnlsParams {
    int64_t n, m, ldM, ldX, ldY;
    const double *M;
    const uint32_t *Mlo;   // 4-byte copy of M (FP32, or BF16 hi << 16 | BF16 lo), same layout
    int prec;              // nmf_gram_precision of the two streaming kernels
    double *X, *Y;
    uint32_t *xmask, *ymask;
    double *bx_part;   // [Sx][K][ldX]  split partials of B_X = M Y^T
    double *by_part;   // [Sy][K][ldY]  split partials of B_Y = X^T M (as B_Y^T)
    double *gx_part;   // [Bx][K*K]     block partials of G_X = X^T X (new X)
    double *gy_part;   // [By][K*K]     block partials of G_Y = Y Y^T (new Y)
    double *xstat;     // [Bx][NST]
    double *ystat;     // [By][NST]
    unsigned *cnt_fin; // [4]
    DevStatus *st;
    int Sx, Tn, xcols; // X stream: Tn row tiles x Sx column splits of xcols columns
    int Sy, Tm, yrows; // Y stream: Tm column tiles x Sy row splits of yrows rows
    int Bx, By;        // row / column blocks of 256 (stage-2 kernels): ceil(n / 256), ceil(m / 256)
    int Nx, Ny;        // stage-1 NNLS blocks: ceil(n / nnls_threads(K)), ceil(m / nnls_threads(K))
    int Wx, Wy;        // waves of the stage-1 NNLS kernels: ceil(n / 64), ceil(m / 64)
    int fx, fy;        // 1: the half is one kernel (k_xfused / k_yfused) whose tile's last
                       // split to finish solves the tile; 0: stream kernel + NNLS kernel
    int Rx, Ry;        // statistics / Gram records of the X- and Y-half: Wx and Wy, or Tn
                       // and Tm when the half is one kernel
    unsigned *tile_cnt; // [Tn + Tm_max] arrival counters of the one-kernel halves' tiles
    int mode;          // X: 0 = solve, 1 = measure E only; Y: 0 = sweep, 2 = appended columns
    // passive-set grouping of the first solve (nmf_set_nnls_grouping)
    int grouped;       // 1: the NNLS kernels try the table of their half first
    int gcap;          // slots of the table: min(2^K, 2048)
    uint8_t *gpresent; // [2^K] sets present in this half (cleared by k_gnumber)
    int *gslot;        // [2^K] slot of each present set, -1 past gcap
    uint32_t *gmask;   // [gcap] set of each slot
    int *gcount;       // slots in use
    double *gtab;      // [gcap][K][K] (G_PP)^-1, zero outside P x P (NaN if G_PP broke down)
};

// Launchers (anls.hip).  All enqueue on `s` and return hipSuccess or an error.
hipError_t launch_xhalf(int K, const AnlsParams &p, hipStream_t s);   // k_xstream + k_xnnls
hipError_t launch_yhalf(int K, const AnlsParams &p, hipStream_t s);   // k_ystream + k_ynnls
// The four stage-1 steps; e0 / e1 (may be null) are recorded by the dispatch
// itself at the start and the end of the kernel.  A half run as one kernel
// (fx / fy) is launched by its stream launcher; its NNLS launcher then does
// nothing and records nothing.
hipError_t launch_xstream(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
hipError_t launch_xnnls(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_ystream(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
hipError_t launch_ynnls(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_measure_finish(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_gram_y_init(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_gram_x_init(int K, const AnlsParams &p, hipStream_t s);
hipError_t launch_objective(int K, const AnlsParams &p, double *part, int nblk, hipStream_t s);
hipError_t launch_check_finite(const double *M, int64_t n, int64_t m, int64_t ldM, double *part,
                               int nblk, hipStream_t s);
hipError_t launch_factor_in(int K, const double *src_x, const double *src_y, const AnlsParams &p,
                            unsigned *bad, hipStream_t s);
hipError_t launch_factor_out(int K, const AnlsParams &p, double *dst_x, double *dst_y, hipStream_t s);
hipError_t launch_make_lowprec(const AnlsParams &p, int64_t j0, int64_t j1, hipStream_t s);
// Re-arms the stage-1 stop rule: converged = 0 and a budget of `budget` more sweeps.
hipError_t launch_rearm(DevStatus *st, int budget, hipStream_t s);
// out[2q] = converged, out[2q+1] = sweeps of the problem of table[q], q < count.
hipError_t launch_batch_poll(const AnlsParams *table, int count, long long *out, hipStream_t s);
// The table of the grouped first solves of one half (yhalf 0: X, 1: Y),
// enqueued by launch_xnnls / launch_ynnls before the solve kernel when
// p.grouped is set.
hipError_t launch_group_table(int K, const AnlsParams &p, int yhalf, hipStream_t s);
hipError_t launch_copy_columns_warm(int K, const AnlsParams &p, int64_t j_from, int64_t j0,
                                    int64_t j1, hipStream_t s);

// A group of problems sharing K and precision, launched as one flattened grid
// per stage-1 kernel.  Device arrays: table[count] and off[NBK][count + 1]
// (block prefix sums of the split X stream, row NNLS, split Y stream, column
// NNLS, fused X half and fused Y half; a problem has blocks in either the
// split or the fused kernels of a half).
constexpr int NBK = 6;   // flattened kernels per batched sweep
struct BatchGroup {
    const AnlsParams *table;
    const int *off;
    int count;
    int blocks[6];
    AnlsParams single;   // host copy used when count == 1 (plain launches, no table lookup)
};
hipError_t launch_batch_sweep(int K, int prec, const BatchGroup &g, hipStream_t s);

int yhalf_cols(int K);   // columns per Y-stream tile, J = YVALS / K

}  // namespace nmfk
