// Stage 2 of the two-stage NMF: the transition (eq. (21)-(25)) and the line-
// search primal-dual interior-point method of Alg. 2 / Alg. 3, on the device.
//
// Newton system.  The reduced system eq. (12) is solved by the route of
// Sec. III-B: Q1bar = P^T P block by block (one k x k Cholesky per row of X),
// then the Schur complement eq. (20)
//     S = Q2bar - (Cbar P^-1)(Cbar P^-1)^T,
// whose (j, l) block is  delta_jl Q2bar_j - sum_i c_ijl X_i^T X_i  with
// c_ijl = Y_j^T Q1bar_i^-1 Y_l = Z_i[:, j] . Z_i[:, l],  Z_i = L_i^-1 Y  (the
// rank-one structure of the blocks of Cbar, Sec. III-B).  With the exact
// Hessian (eq. (27), flag = 1) block (j, i) of C gains (XY - M)_ij I and the
// sum gains three terms (R_il X_ia w_ij[b] + R_ij w_il[a] X_ib + R_ij R_il
// Q1bar_i^-1[a][b], w_ij = Q1bar_i^-1 Y_j).
// The products with Cbar that the right-hand side and the back substitution
// need reduce to k x k matrices:  (Cbar v)_j = (X^T V) Y_j  and
// (Cbar^T dy)_i = X_i (dY Y^T);  the exact-Hessian parts are one pass over M
// with the residual formed on the fly.
//
// Line search.  With R0 = XY - M, A = dX Y + X dY, B = dX dY, the objective
// along the step is 1/2 ||R0 + a A + a^2 B||^2, a quartic whose six
// coefficients come from one pass over M; the barrier terms of phi for a batch
// of trial steps a = a1max / 2^t come from one pass over (x, y).
//
// Dense linear algebra (dense.hip).  The unknowns dy are ordered component-
// major (index a*m + j); the Gauss-Newton S is formed on FP64 matrix cores,
// factored by 64-wide block columns (one launch per block column) and solved
// by two single-launch blocked triangular solves.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstddef>
#include <vector>

#include "dense.h"
#include "device_util.h"
#include "ipm.h"

namespace nmfk {

constexpr int PRS = KMAX * KMAX;   // stride of block records in `part`
// Slots of the scalar block's `out`: the direction's slope and step limits,
// the line-search quartic and first barrier batch, the Armijo choice made on
// the device ([0] accepted, [1] a1, [2] a2, [3] backtracks), the KKT sums
// of the point it leads to, and the predictor's complementarity sum.
constexpr int OUT_DIR = 0, OUT_QUART = 8, OUT_BAR = 16;
constexpr int OUT_SEL = OUT_BAR + NTRIAL, OUT_KKT = OUT_SEL + 4, OUT_AFF = OUT_KKT + 4;
static_assert(OUT_AFF + 1 <= 4 * PARTW, "the finish outputs fit the scalar block");
constexpr int CB = 64;             // dense Cholesky / triangular-solve tile
constexpr int TJ = 16;             // Schur tile: 16 x 16 (j, l) pairs
constexpr int ZRB = 8;             // rows per block of the Z kernel

struct IpmArgs {
    double *r, *s, *dx, *dy, *dr, *ds, *gx, *gy, *V, *tX, *tY, *Lq, *Z, *S, *vec, *vec2, *part;
    IpmScal *sc;
    int64_t ldS, N;
};

static IpmArgs args_of(const IpmState &s) {
    IpmArgs a;
    a.r = s.r; a.s = s.s; a.dx = s.dx; a.dy = s.dy; a.dr = s.dr; a.ds = s.ds;
    a.gx = s.gx; a.gy = s.gy; a.V = s.V; a.tX = s.tX; a.tY = s.tY; a.Lq = s.Lq;
    a.Z = s.Z; a.S = s.S; a.vec = s.vec; a.vec2 = s.vec2; a.part = s.part; a.sc = s.sc;
    a.ldS = s.ldS;
    a.N = 0;
    return a;
}

// Sums V values given by fn(idx) (compile-time idx after unrolling) over the
// block; value q lands in out[q].  lds holds blockDim doubles.
template <int V, class F>
__device__ __forceinline__ void block_reduce_fn(F &&fn, double *out, double *lds) {
    constexpr int NPASS = (V + YVALS - 1) / YVALS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        double v[YVALS];
#pragma unroll
        for (int q = 0; q < YVALS; ++q) v[q] = (pass * YVALS + q < V) ? fn(pass * YVALS + q) : 0.0;
        lds[w * YVALS + lane] = wave_transpose_reduce(v, lane);
        __syncthreads();
        const int idx = pass * YVALS + (int)threadIdx.x;
        if ((int)threadIdx.x < YVALS && idx < V) {
            double sum = lds[threadIdx.x];
            for (int ww = 1; ww < (int)blockDim.x / 64; ++ww) sum += lds[ww * YVALS + threadIdx.x];
            out[idx] = sum;
        }
        __syncthreads();
    }
}

// out[q] = sum (or min, bit q of minmask) over nblk records part[b*stride + q],
// by NTHR threads: thread (q, g) reduces records g, g + G, ... (G = NTHR /
// nval), then thread q reduces the G partial results in order.
__device__ __forceinline__ void finish_body(const double *part, int stride, int nblk, int nval, unsigned minmask,
                                            double *out, double *scr) {
    const int G = NTHR / nval;
    const int q = threadIdx.x % nval, g = threadIdx.x / nval;
    const bool mn = (minmask >> q) & 1u;
    if (g < G) {
        double acc = mn ? INFINITY : 0.0;
        for (int t = g; t < nblk; t += G) {
            const double v = part[(size_t)t * stride + q];
            acc = mn ? (v < acc ? v : acc) : acc + v;
        }
        scr[threadIdx.x] = acc;
    }
    __syncthreads();
    if ((int)threadIdx.x < nval) {
        double acc = scr[threadIdx.x];
        for (int gg = 1; gg < G; ++gg) {
            const double v = scr[gg * nval + threadIdx.x];
            acc = mn ? (v < acc ? v : acc) : acc + v;
        }
        out[threadIdx.x] = acc;
    }
}

__global__ __launch_bounds__(NTHR) void k_finish(const double *part, int stride, int nblk, int nval,
                                                 unsigned minmask, double *out) {
    __shared__ double scr[NTHR];
    finish_body(part, stride, nblk, nval, minmask, out, scr);
}

// The same reduction done by the last block of the kernel that wrote the
// records (one launch fewer); out == nullptr: none.  cnt counts the arriving
// blocks and wraps to zero for the next kernel.
struct FinArgs {
    const double *part;
    double *out;
    unsigned *cnt;
    int stride, nblk, nval;
    unsigned minmask;
};

// Called by every thread of a kernel launched with NTHR threads per block,
// after the block's record is written (by wave 0, which fences it).
__device__ __forceinline__ void finish_last(const FinArgs &f) {
    if (!f.out) return;
    __shared__ unsigned flag;
    __shared__ double scr[NTHR];
    if (!last_arrival(f.cnt, gridDim.x * gridDim.y, &flag)) return;
    finish_body(f.part, f.stride, f.nblk, f.nval, f.minmask, f.out, scr);
}

// out[a*ld + e] = sum_s part[(s*K + a)*ld + e], e < count; component a =
// blockIdx.y (one thread per entry, the splits summed in order).
__global__ __launch_bounds__(NTHR) void k_sum_splits(const double *part, int S, int K, int64_t ld, int64_t count,
                                                     double *out) {
    const int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    const int a = (int)blockIdx.y;
    if (e >= count) return;
    double v = 0.0;
    for (int s = 0; s < S; ++s) v += part[((int64_t)s * K + a) * ld + e];
    out[(int64_t)a * ld + e] = v;
}

// ---------------------------------------------------------------- residual streams
// X side: out_part[split][a][i] = sum_{j in split} R_ij W[a][j], R = XY - M;
// fpart[tile * Sx + split] = the block's share of sum R_ij^2 (if fpart).
template <int K>
__global__ __launch_bounds__(STHR) void k_rstream_x(AnlsParams p, const double *W, double *out_part,
                                                    double *fpart) {
    constexpr int RED = SWAVES * K * XTILE + SWAVES * XTILE;
    constexpr int LDSN = (2 * XCHUNK * K > RED) ? 2 * XCHUNK * K : RED;
    __shared__ double lds[LDSN];
    double *ys = lds, *ws = lds + XCHUNK * K;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)tile * XTILE + lane;
    const int64_t j0 = (int64_t)split * p.xcols;
    const int64_t j1 = min(j0 + (int64_t)p.xcols, p.m);
    const bool row_ok = i < p.n;
    double x[K], acc[K], f = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        x[a] = row_ok ? p.X[(int64_t)a * p.ldX + i] : 0.0;
        acc[a] = 0.0;
    }
    for (int64_t c0 = j0; c0 < j1; c0 += XCHUNK) {
        const int nc = (int)min((int64_t)XCHUNK, j1 - c0);
        __syncthreads();
        for (int q = threadIdx.x; q < nc * K; q += STHR) {
            const int jj = q / K, a = q - jj * K;
            ys[q] = p.Y[(int64_t)a * p.ldY + c0 + jj];
            ws[q] = W[(int64_t)a * p.ldY + c0 + jj];
        }
        __syncthreads();
        const double *mp = p.M + c0 * p.ldM + (row_ok ? i : 0);
        for (int jb = w; jb < nc; jb += 8 * SWAVES) {
            double mv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int jj = jb + t * SWAVES;
                mv[t] = (jj < nc && row_ok) ? mp[(int64_t)jj * p.ldM] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int jj = jb + t * SWAVES;
                if (jj < nc) {
                    double rr = -mv[t];
#pragma unroll
                    for (int a = 0; a < K; ++a) rr = fma(x[a], ys[jj * K + a], rr);
                    if (!row_ok) rr = 0.0;
#pragma unroll
                    for (int a = 0; a < K; ++a) acc[a] = fma(rr, ws[jj * K + a], acc[a]);
                    f = fma(rr, rr, f);
                }
            }
        }
    }
    __syncthreads();
    double *red = lds, *fred = lds + SWAVES * K * XTILE;
#pragma unroll
    for (int a = 0; a < K; ++a) red[(w * K + a) * XTILE + lane] = acc[a];
    fred[w * XTILE + lane] = f;
    __syncthreads();
    if (w == 0) {
        if (row_ok) {
#pragma unroll
            for (int a = 0; a < K; ++a) {
                double v = red[a * XTILE + lane];
#pragma unroll
                for (int ww = 1; ww < SWAVES; ++ww) v += red[(ww * K + a) * XTILE + lane];
                out_part[((int64_t)split * K + a) * p.ldX + i] = v;
            }
        }
        if (fpart) {
            double fl = fred[lane];
#pragma unroll
            for (int ww = 1; ww < SWAVES; ++ww) fl += fred[ww * XTILE + lane];
#pragma unroll
            for (int h = 32; h >= 1; h >>= 1) fl += __shfl_xor(fl, h, 64);
            if (lane == 0) fpart[(int64_t)tile * p.Sx + split] = fl;
        }
    }
}

// Y side: out_part[split][a][j] = sum_{i in split} R_ij Vm[a][i].
template <int K>
__global__ __launch_bounds__(STHR) void k_rstream_y(AnlsParams p, const double *Vm, double *out_part) {
    constexpr int J = YVALS / K;
    __shared__ double red[SWAVES * YVALS];
    __shared__ double yts[J * K];
    const int ct = blockIdx.x, split = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t jb = (int64_t)ct * J;
    const int nj = (int)min((int64_t)J, p.m - jb);
    const int64_t r0 = (int64_t)split * p.yrows;
    const int64_t r1 = min(r0 + (int64_t)p.yrows, p.n);
    if ((int)threadIdx.x < J * K) {
        const int jj = threadIdx.x / K, a = threadIdx.x - jj * K;
        yts[threadIdx.x] = jj < nj ? p.Y[(int64_t)a * p.ldY + jb + jj] : 0.0;
    }
    __syncthreads();
    double v[YVALS];
#pragma unroll
    for (int q = 0; q < YVALS; ++q) v[q] = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += STHR) {
        double x[K], vm[K], mv[J];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            x[a] = p.X[(int64_t)a * p.ldX + i];
            vm[a] = Vm[(int64_t)a * p.ldX + i];
        }
        const double *mp = p.M + jb * p.ldM + i;
#pragma unroll
        for (int jj = 0; jj < J; ++jj) mv[jj] = (jj < nj) ? mp[(int64_t)jj * p.ldM] : 0.0;
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
            double rr = -mv[jj];
#pragma unroll
            for (int a = 0; a < K; ++a) rr = fma(x[a], yts[jj * K + a], rr);
#pragma unroll
            for (int a = 0; a < K; ++a) v[jj * K + a] = fma(rr, vm[a], v[jj * K + a]);
        }
    }
    red[w * YVALS + lane] = wave_transpose_reduce(v, lane);
    __syncthreads();
    if ((int)threadIdx.x < nj * K) {
        double s = red[threadIdx.x];
#pragma unroll
        for (int ww = 1; ww < SWAVES; ++ww) s += red[ww * YVALS + threadIdx.x];
        const int jj = threadIdx.x / K, a = threadIdx.x - jj * K;
        out_part[((int64_t)split * K + a) * p.ldY + jb + jj] = s;
    }
}

// Block partials of sum_e A_e B_e^T (K x K, row-major a*K + b) over
// e < count, A and B component-major with leading dimension ld.
template <int K>
__global__ __launch_bounds__(NTHR) void k_outer(const double *A, const double *B, int64_t ld, int64_t count,
                                                double *part, FinArgs fa) {
    __shared__ double lds[NTHR];
    const int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    double a[K], b[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        a[q] = e < count ? A[(int64_t)q * ld + e] : 0.0;
        b[q] = e < count ? B[(int64_t)q * ld + e] : 0.0;
    }
    block_reduce_fn<K * K>([&](int idx) { return a[idx / K] * b[idx % K]; }, part + (size_t)blockIdx.x * PRS,
                           lds);
    finish_last(fa);
}

// ---------------------------------------------------------------- point kernels
// Blocks [0, Bx) cover rows (x, r, gx), blocks [Bx, Bx + By) columns (y, s, gy).
struct Side {
    const double *v, *d, *g;
    double *dual;
    int64_t ld, count, e;
    bool ok;
};

template <int K>
__device__ __forceinline__ Side side_of(const AnlsParams &p, const IpmArgs &ia, bool use_dir) {
    Side sd;
    const int b = blockIdx.x;
    if (b < p.Bx) {
        sd.v = p.X; sd.d = use_dir ? ia.dx : nullptr; sd.g = ia.gx; sd.dual = ia.r;
        sd.ld = p.ldX; sd.count = p.n; sd.e = (int64_t)b * NTHR + threadIdx.x;
    } else {
        sd.v = p.Y; sd.d = use_dir ? ia.dy : nullptr; sd.g = ia.gy; sd.dual = ia.s;
        sd.ld = p.ldY; sd.count = p.m; sd.e = (int64_t)(b - p.Bx) * NTHR + threadIdx.x;
    }
    sd.ok = sd.e < sd.count;
    return sd;
}

// KKT sums at the current point: [0] sum (g - dual)^2, [1] sum (dual v)^2,
// [2] sum (dual v - mu)^2, [3] sum dual v.
template <int K>
__global__ __launch_bounds__(NTHR) void k_kkt(AnlsParams p, IpmArgs ia, double mu, FinArgs fa) {
    __shared__ double lds[NTHR];
    const Side sd = side_of<K>(p, ia, false);
    double s1 = 0.0, c0 = 0.0, cm = 0.0, sr = 0.0;
    if (sd.ok) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * sd.ld + sd.e;
            const double gd = sd.g[o] - sd.dual[o];
            const double c = sd.dual[o] * sd.v[o];
            s1 = fma(gd, gd, s1);
            c0 = fma(c, c, c0);
            cm = fma(c - mu, c - mu, cm);
            sr += c;
        }
    }
    const double vals[4] = {s1, c0, cm, sr};
    block_reduce_fn<4>([&](int idx) { return vals[idx]; }, ia.part + (size_t)blockIdx.x * PRS, lds);
    finish_last(fa);
}

// Transition helpers.  mode 0: [0] = -max v ; mode 1: [0] = -max |g|, per side
// in its own slot ([0] rows, [1] columns), so that a min-finish gives both.
template <int K>
__global__ __launch_bounds__(NTHR) void k_maxes(AnlsParams p, IpmArgs ia, int mode) {
    __shared__ double lds[NTHR];
    const Side sd = side_of<K>(p, ia, false);
    double mx = -INFINITY;
    if (sd.ok) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * sd.ld + sd.e;
            const double v = mode == 0 ? sd.v[o] : fabs(sd.g[o]);
            mx = v > mx ? v : mx;
        }
    }
    lds[threadIdx.x] = mx;
    __syncthreads();
    for (int h = NTHR / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] = lds[threadIdx.x + h] > lds[threadIdx.x] ? lds[threadIdx.x + h] : lds[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool rows = (int)blockIdx.x < p.Bx;
        double *rec = ia.part + (size_t)blockIdx.x * PRS;
        rec[0] = rows ? -lds[0] : INFINITY;
        rec[1] = rows ? INFINITY : -lds[0];
    }
}

template <int K>
__global__ __launch_bounds__(NTHR) void k_clamp(AnlsParams p, double lo) {
    const int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    if (e < p.n) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double *q = p.X + (int64_t)a * p.ldX + e;
            *q = *q > lo ? *q : lo;
        }
    }
    if (e < p.m) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double *q = p.Y + (int64_t)a * p.ldY + e;
            *q = *q > lo ? *q : lo;
        }
    }
}

// r = rv, s = sv everywhere; records [0] sum x (rows), [1] sum y (columns).
template <int K>
__global__ __launch_bounds__(NTHR) void k_fill_duals(AnlsParams p, IpmArgs ia, double rv, double sv) {
    __shared__ double lds[NTHR];
    const Side sd = side_of<K>(p, ia, false);
    const bool rows = (int)blockIdx.x < p.Bx;
    double sum = 0.0;
    if (sd.ok) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * sd.ld + sd.e;
            sd.dual[o] = rows ? rv : sv;
            sum += sd.v[o];
        }
    }
    const double vals[2] = {rows ? sum : 0.0, rows ? 0.0 : sum};
    block_reduce_fn<2>([&](int idx) { return vals[idx]; }, ia.part + (size_t)blockIdx.x * PRS, lds);
}

// ---------------------------------------------------------------- direction
// Per row i: the Cholesky factor L_i of Q1bar_i = Y Y^T + rho I + Diag(r_i / x_i)
// (packed lower, then 1/diag) and V_i = Q1bar_i^-1 b1_i with b1 = -(graX - mu/x).
template <int K>
__global__ __launch_bounds__(NTHR) void k_factor(AnlsParams p, IpmArgs ia, double mu, double rho) {
    constexpr int NL = K * (K + 1) / 2;
    __shared__ double G[K * K];
    for (int q = threadIdx.x; q < K * K; q += NTHR) G[q] = ia.sc->GY[q];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    if (i >= p.n) return;
    double L[NL], inv[K], x[K], b1[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int64_t o = (int64_t)a * p.ldX + i;
        x[a] = p.X[o];
        b1[a] = -(ia.gx[o] - mu / x[a]);
    }
#pragma unroll
    for (int r = 0; r < K; ++r) {
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            double v = G[r * K + c];
            if (r == c) v += rho + ia.r[(int64_t)r * p.ldX + i] / x[r];
#pragma unroll
            for (int q = 0; q < c; ++q) v -= L[r * (r + 1) / 2 + q] * L[c * (c + 1) / 2 + q];
            if (r == c) {
                const double d = sqrt(v);
                L[r * (r + 1) / 2 + r] = d;
                inv[r] = 1.0 / d;
            } else {
                L[r * (r + 1) / 2 + c] = v * inv[c];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) ia.Lq[(int64_t)q * p.ldX + i] = L[q];
#pragma unroll
    for (int a = 0; a < K; ++a) ia.Lq[(int64_t)(NL + a) * p.ldX + i] = inv[a];
    // V_i = L^-T L^-1 b1
    double t[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        double v = b1[r];
#pragma unroll
        for (int q = 0; q < r; ++q) v -= L[r * (r + 1) / 2 + q] * t[q];
        t[r] = v * inv[r];
    }
#pragma unroll
    for (int r = K - 1; r >= 0; --r) {
        double v = t[r];
#pragma unroll
        for (int q = r + 1; q < K; ++q) v -= L[q * (q + 1) / 2 + r] * t[q];
        t[r] = v * inv[r];
    }
#pragma unroll
    for (int a = 0; a < K; ++a) ia.V[(int64_t)a * p.ldX + i] = t[a];
}

// Z_i = L_i^-1 Y for ZRB rows per block: Z[(i*KP + c)*ldY + j], KP = K
// rounded up to a multiple of 4, zero for c >= K and for j >= m.
template <int K>
__global__ __launch_bounds__(NTHR) void k_zmat(AnlsParams p, IpmArgs ia) {
    constexpr int NL = K * (K + 1) / 2;
    __shared__ double Ls[ZRB][NL + K];
    const int64_t i0 = (int64_t)blockIdx.x * ZRB;
    for (int q = threadIdx.x; q < ZRB * (NL + K); q += NTHR) {
        const int rr = q / (NL + K), c = q - rr * (NL + K);
        const int64_t i = i0 + rr;
        Ls[rr][c] = i < p.n ? ia.Lq[(int64_t)c * p.ldX + i] : 1.0;
    }
    __syncthreads();
    const int nr = (int)min((int64_t)ZRB, p.n - i0);
    constexpr int KP = zpad(K);
    // every column up to ldY and components up to KP: the padding is 0
    for (int64_t j = threadIdx.x; j < p.ldY; j += NTHR) {
        double y[K];
#pragma unroll
        for (int a = 0; a < K; ++a) y[a] = j < p.m ? p.Y[(int64_t)a * p.ldY + j] : 0.0;
        for (int rr = 0; rr < nr; ++rr) {
            double z[K];
#pragma unroll
            for (int r = 0; r < K; ++r) {
                double v = y[r];
#pragma unroll
                for (int q = 0; q < r; ++q) v -= Ls[rr][r * (r + 1) / 2 + q] * z[q];
                z[r] = v * Ls[rr][NL + r];
            }
#pragma unroll
            for (int c = 0; c < KP; ++c) ia.Z[((i0 + rr) * KP + c) * p.ldY + j] = c < K ? z[c] : 0.0;
        }
    }
}

// Right-hand side of eq. (20): rhs_j = b2_j - (X^T V) Y_j [- (R^T V)_j], b2 = -(graY - mu/y).
template <int K, bool EXACT>
__global__ __launch_bounds__(NTHR) void k_rhs(AnlsParams p, IpmArgs ia, double mu) {
    __shared__ double T[K * K];
    for (int q = threadIdx.x; q < K * K; q += NTHR) T[q] = ia.sc->XtV[q];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    const int64_t N = p.m * K, Np = (N + CB - 1) / CB * CB;
    if (j < Np - N) ia.vec[N + j] = 0.0;   // the identity padding of S solves to 0
    if (j >= p.m) return;
    double y[K];
#pragma unroll
    for (int a = 0; a < K; ++a) y[a] = p.Y[(int64_t)a * p.ldY + j];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double v = -(ia.gy[(int64_t)a * p.ldY + j] - mu / y[a]);
#pragma unroll
        for (int b = 0; b < K; ++b) v -= T[a * K + b] * y[b];
        if (EXACT) v -= ia.tY[(int64_t)a * p.ldY + j];
        ia.vec[a * p.m + j] = v;
    }
}

// Column side after the Schur solve: dY from the solution, ds, and the
// records [0] slope part, [1] alpha1 candidate, [2] alpha2 candidate.
template <int K>
__global__ __launch_bounds__(NTHR) void k_post_y(AnlsParams p, IpmArgs ia, double mu, double tau, int recbase) {
    __shared__ double lds[NTHR];
    const int64_t j = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    double slope = 0.0, a1 = INFINITY, a2 = INFINITY;
    if (j < p.m) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * p.ldY + j;
            const double d = ia.vec2[a * p.m + j];
            const double y = p.Y[o], s = ia.s[o];
            ia.dy[o] = d;
            const double dsv = mu / y - s - (s / y) * d;
            ia.ds[o] = dsv;
            slope = fma(d, ia.gy[o] - mu / y, slope);
            if (d < 0.0) { const double c = -tau * y / d; a1 = c < a1 ? c : a1; }
            if (dsv < 0.0) { const double c = -tau * s / dsv; a2 = c < a2 ? c : a2; }
        }
    }
    a1 = wave_min(a1);
    a2 = wave_min(a2);
    const double vals[1] = {slope};
    double *rec = ia.part + (size_t)(recbase + blockIdx.x) * PRS;
    block_reduce_fn<1>([&](int idx) { return vals[idx]; }, rec, lds);
    __shared__ double mins[2][NTHR / 64];
    if ((threadIdx.x & 63) == 0) {
        mins[0][threadIdx.x >> 6] = a1;
        mins[1][threadIdx.x >> 6] = a2;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double m = mins[threadIdx.x][0];
        for (int w = 1; w < NTHR / 64; ++w) m = mins[threadIdx.x][w] < m ? mins[threadIdx.x][w] : m;
        rec[1 + threadIdx.x] = m;
    }
}

// Row side: dx_i = V_i - Q1bar_i^-1 (X_i (dY Y^T) [+ (R dY^T)_i]), dr, and the
// same three records.
template <int K, bool EXACT>
__global__ __launch_bounds__(NTHR) void k_post_x(AnlsParams p, IpmArgs ia, double mu, double tau, int recbase,
                                                 FinArgs fa) {
    constexpr int NL = K * (K + 1) / 2;
    __shared__ double T[K * K];
    __shared__ double lds[NTHR];
    for (int q = threadIdx.x; q < K * K; q += NTHR) T[q] = ia.sc->T[q];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    double slope = 0.0, a1 = INFINITY, a2 = INFINITY;
    if (i < p.n) {
        double x[K], u[K];
#pragma unroll
        for (int a = 0; a < K; ++a) x[a] = p.X[(int64_t)a * p.ldX + i];
#pragma unroll
        for (int b = 0; b < K; ++b) {
            double v = EXACT ? ia.tX[(int64_t)b * p.ldX + i] : 0.0;
#pragma unroll
            for (int a = 0; a < K; ++a) v = fma(x[a], T[a * K + b], v);
            u[b] = v;
        }
        // w = L^-T L^-1 u
#pragma unroll
        for (int r = 0; r < K; ++r) {
            double v = u[r];
#pragma unroll
            for (int q = 0; q < r; ++q) v -= ia.Lq[(int64_t)(r * (r + 1) / 2 + q) * p.ldX + i] * u[q];
            u[r] = v * ia.Lq[(int64_t)(NL + r) * p.ldX + i];
        }
#pragma unroll
        for (int r = K - 1; r >= 0; --r) {
            double v = u[r];
#pragma unroll
            for (int q = r + 1; q < K; ++q) v -= ia.Lq[(int64_t)(q * (q + 1) / 2 + r) * p.ldX + i] * u[q];
            u[r] = v * ia.Lq[(int64_t)(NL + r) * p.ldX + i];
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * p.ldX + i;
            const double d = ia.V[o] - u[a];
            const double r = ia.r[o];
            ia.dx[o] = d;
            const double drv = mu / x[a] - r - (r / x[a]) * d;
            ia.dr[o] = drv;
            slope = fma(d, ia.gx[o] - mu / x[a], slope);
            if (d < 0.0) { const double c = -tau * x[a] / d; a1 = c < a1 ? c : a1; }
            if (drv < 0.0) { const double c = -tau * r / drv; a2 = c < a2 ? c : a2; }
        }
    }
    a1 = wave_min(a1);
    a2 = wave_min(a2);
    const double vals[1] = {slope};
    double *rec = ia.part + (size_t)(recbase + blockIdx.x) * PRS;
    block_reduce_fn<1>([&](int idx) { return vals[idx]; }, rec, lds);
    __shared__ double mins[2][NTHR / 64];
    if ((threadIdx.x & 63) == 0) {
        mins[0][threadIdx.x >> 6] = a1;
        mins[1][threadIdx.x >> 6] = a2;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double m = mins[threadIdx.x][0];
        for (int w = 1; w < NTHR / 64; ++w) m = mins[threadIdx.x][w] < m ? mins[threadIdx.x][w] : m;
        rec[1 + threadIdx.x] = m;
    }
    finish_last(fa);
}

// ---------------------------------------------------------------- line search
// Six inner products over M: [0] <R0,R0>, [1] <R0,A>, [2] <A,A>, [3] <R0,B>,
// [4] <A,B>, [5] <B,B>, R0 = XY - M, A = dX Y + X dY, B = dX dY.
template <int K>
__global__ __launch_bounds__(STHR) void k_ls_quartic(AnlsParams p, IpmArgs ia, double *lspart) {
    __shared__ double lds[2 * XCHUNK * K > STHR ? 2 * XCHUNK * K : STHR];
    double *ys = lds, *dys = lds + XCHUNK * K;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)tile * XTILE + lane;
    const int64_t j0 = (int64_t)split * p.xcols;
    const int64_t j1 = min(j0 + (int64_t)p.xcols, p.m);
    const bool row_ok = i < p.n;
    double x[K], dx[K], c[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < K; ++a) {
        x[a] = row_ok ? p.X[(int64_t)a * p.ldX + i] : 0.0;
        dx[a] = row_ok ? ia.dx[(int64_t)a * p.ldX + i] : 0.0;
    }
    for (int64_t c0 = j0; c0 < j1; c0 += XCHUNK) {
        const int nc = (int)min((int64_t)XCHUNK, j1 - c0);
        __syncthreads();
        for (int q = threadIdx.x; q < nc * K; q += STHR) {
            const int jj = q / K, a = q - jj * K;
            ys[q] = p.Y[(int64_t)a * p.ldY + c0 + jj];
            dys[q] = ia.dy[(int64_t)a * p.ldY + c0 + jj];
        }
        __syncthreads();
        if (row_ok) {
            const double *mp = p.M + c0 * p.ldM + i;
            for (int jj = w; jj < nc; jj += SWAVES) {
                const double mv = mp[(int64_t)jj * p.ldM];
                double R0 = -mv, A = 0.0, B = 0.0;
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const double y = ys[jj * K + a], dy = dys[jj * K + a];
                    R0 = fma(x[a], y, R0);
                    A = fma(dx[a], y, A);
                    A = fma(x[a], dy, A);
                    B = fma(dx[a], dy, B);
                }
                c[0] = fma(R0, R0, c[0]);
                c[1] = fma(R0, A, c[1]);
                c[2] = fma(A, A, c[2]);
                c[3] = fma(R0, B, c[3]);
                c[4] = fma(A, B, c[4]);
                c[5] = fma(B, B, c[5]);
            }
        }
    }
    __syncthreads();
    block_reduce_fn<6>([&](int idx) { return c[idx]; }, lspart + ((int64_t)tile * p.Sx + split) * 8, lds);
}

// Barrier sums for NTRIAL steps a_t = a_base / 2^t:
// record[t] = sum over the block's entries of log1p(a_t d / v).
// Trials t = blockIdx.y * LS_TG + (0 .. LS_TG - 1), step a_base 2^-t (exact
// scalings); block b writes trial t of its entries to part[b * PRS + t].
constexpr int LS_TG = 2;
static_assert(NTRIAL % LS_TG == 0, "trial groups");
template <int K>
__global__ __launch_bounds__(NTHR) void k_ls_barrier(AnlsParams p, IpmArgs ia, const double *a1dev, double a_base,
                                                     FinArgs fa) {
    __shared__ double lds[NTHR];
    // first batch: a_base = min(a1, 1) from the direction's step limit on the device
    if (a1dev) a_base = a1dev[0] < 1.0 ? a1dev[0] : 1.0;
    const int t0 = (int)blockIdx.y * LS_TG;
    const Side sd = side_of<K>(p, ia, true);
    double acc[LS_TG];
#pragma unroll
    for (int t = 0; t < LS_TG; ++t) acc[t] = 0.0;
    if (sd.ok) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * sd.ld + sd.e;
            const double q = sd.d[o] / sd.v[o];
            double at = ldexp(a_base, -t0);
#pragma unroll
            for (int t = 0; t < LS_TG; ++t) {
                acc[t] += log1p(at * q);
                at *= 0.5;
            }
        }
    }
    block_reduce_fn<LS_TG>([&](int idx) { return acc[idx]; }, ia.part + (size_t)blockIdx.x * PRS + t0, lds);
    finish_last(fa);
}

// sel != nullptr: the step comes from the device's Armijo choice (sel[0] = 0:
// none accepted, the point is left as it is).
template <int K>
__global__ __launch_bounds__(NTHR) void k_update(AnlsParams p, IpmArgs ia, double a1, double a2, const double *sel) {
    if (sel) {
        if (sel[0] == 0.0) return;
        a1 = sel[1];
        a2 = sel[2];
    }
    const int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    if (e < p.n) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * p.ldX + e;
            p.X[o] += a1 * ia.dx[o];
            ia.r[o] += a2 * ia.dr[o];
        }
    }
    if (e < p.m) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * p.ldY + e;
            p.Y[o] += a1 * ia.dy[o];
            ia.s[o] += a2 * ia.ds[o];
        }
    }
}

// The first batch of the Armijo rule of eq. (13) on the device, with the
// arithmetic of the host's line search (no contraction): the step limits and
// slope of the direction (out[OUT_DIR..]), the quartic (out[OUT_QUART..]) and
// the barrier sums of the first NTRIAL trials (out[OUT_BAR..]); writes the
// choice to out[OUT_SEL..].  Nothing is accepted when the factorisation that
// produced the direction failed.
__global__ void k_armijo(IpmScal *sc, double mu, double eta, int maxb, int formed) {
#pragma clang fp contract(off)
    if (threadIdx.x != 0) return;
    const double *h = sc->out;
    double *sel = sc->out + OUT_SEL;
    sel[0] = 0.0;
    sel[1] = 0.0;
    sel[2] = 0.0;
    sel[3] = 0.0;
    if (formed && sc->chol_fail) return;
    const double slope = h[OUT_DIR];
    const double a1 = h[OUT_DIR + 1] < 1.0 ? h[OUT_DIR + 1] : 1.0;
    const double a2 = h[OUT_DIR + 2] < 1.0 ? h[OUT_DIR + 2] : 1.0;
    const double *q = h + OUT_QUART;
    const double *bar = h + OUT_BAR;
    for (int t = 0; t < NTRIAL && t <= maxb; ++t) {
        const double a = a1 / ldexp(1.0, t);
        const double dq = 0.5 * (2.0 * a * q[1] + a * a * (q[2] + 2.0 * q[3]) + 2.0 * a * a * a * q[4] +
                                 a * a * a * a * q[5]);
        const double dphi = dq - mu * bar[t];
        if (dphi <= eta * a * slope) {
            sel[0] = 1.0;
            sel[1] = a;
            sel[2] = a2;
            sel[3] = (double)t;
            return;
        }
    }
}

// Predictor probe, eq. (8): [0] sum (v + a1 d)(dual + a2 ddual).
template <int K>
// adev != nullptr: the step limits are read from the device (adev[0], adev[1]
// capped at 1, as the host caps them).
__global__ __launch_bounds__(NTHR) void k_muaff(AnlsParams p, IpmArgs ia, double a1, double a2, const double *adev,
                                                FinArgs fa) {
    __shared__ double lds[NTHR];
    if (adev) {
        a1 = adev[0] < 1.0 ? adev[0] : 1.0;
        a2 = adev[1] < 1.0 ? adev[1] : 1.0;
    }
    const Side sd = side_of<K>(p, ia, true);
    const double *dd = (int)blockIdx.x < p.Bx ? ia.dr : ia.ds;
    double acc = 0.0;
    if (sd.ok) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int64_t o = (int64_t)a * sd.ld + sd.e;
            acc += (sd.v[o] + a1 * sd.d[o]) * (sd.dual[o] + a2 * dd[o]);
        }
    }
    const double vals[1] = {acc};
    block_reduce_fn<1>([&](int idx) { return vals[idx]; }, ia.part + (size_t)blockIdx.x * PRS, lds);
    finish_last(fa);
}

// Stage-1 masks from the signs (used when the context returns to stage 1).
template <int K>
__global__ __launch_bounds__(NTHR) void k_masks(AnlsParams p) {
    const int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    if (e < p.n) {
        uint32_t P = 0;
#pragma unroll
        for (int a = 0; a < K; ++a)
            if (p.X[(int64_t)a * p.ldX + e] > 0.0) P |= 1u << a;
        p.xmask[e] = P;
    }
    if (e < p.m) {
        uint32_t P = 0;
#pragma unroll
        for (int a = 0; a < K; ++a)
            if (p.Y[(int64_t)a * p.ldY + e] > 0.0) P |= 1u << a;
        p.ymask[e] = P;
    }
}

// Duals out: R as n x K row-major, S as K x m row-major.
template <int K>
__global__ __launch_bounds__(NTHR) void k_duals_out(AnlsParams p, IpmArgs ia, double *R, double *S) {
    const int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    if (R && e < p.n) {
#pragma unroll
        for (int a = 0; a < K; ++a) R[e * K + a] = ia.r[(int64_t)a * p.ldX + e];
    }
    if (S && e < p.m) {
#pragma unroll
        for (int a = 0; a < K; ++a) S[(int64_t)a * p.m + e] = ia.s[(int64_t)a * p.ldY + e];
    }
}

// ================================================================= host side
#define IPM_K_SWITCH(K, CALL)                                \
    switch (K) {                                             \
        case 1: { constexpr int KK = 1; CALL; } break;       \
        case 2: { constexpr int KK = 2; CALL; } break;       \
        case 3: { constexpr int KK = 3; CALL; } break;       \
        case 4: { constexpr int KK = 4; CALL; } break;       \
        case 5: { constexpr int KK = 5; CALL; } break;       \
        case 6: { constexpr int KK = 6; CALL; } break;       \
        case 7: { constexpr int KK = 7; CALL; } break;       \
        case 8: { constexpr int KK = 8; CALL; } break;       \
        case 9: { constexpr int KK = 9; CALL; } break;       \
        case 10: { constexpr int KK = 10; CALL; } break;     \
        case 11: { constexpr int KK = 11; CALL; } break;     \
        case 12: { constexpr int KK = 12; CALL; } break;     \
        case 13: { constexpr int KK = 13; CALL; } break;     \
        case 14: { constexpr int KK = 14; CALL; } break;     \
        case 15: { constexpr int KK = 15; CALL; } break;     \
        case 16: { constexpr int KK = 16; CALL; } break;     \
        default: return hipErrorInvalidValue;                \
    }

#define IPM_KS(K, CALL)                                \
    switch (K) {                                             \
        case 1: { constexpr int KK = 1; CALL; } break;       \
        case 2: { constexpr int KK = 2; CALL; } break;       \
        case 3: { constexpr int KK = 3; CALL; } break;       \
        case 4: { constexpr int KK = 4; CALL; } break;       \
        case 5: { constexpr int KK = 5; CALL; } break;       \
        case 6: { constexpr int KK = 6; CALL; } break;       \
        case 7: { constexpr int KK = 7; CALL; } break;       \
        case 8: { constexpr int KK = 8; CALL; } break;       \
        case 9: { constexpr int KK = 9; CALL; } break;       \
        case 10: { constexpr int KK = 10; CALL; } break;     \
        case 11: { constexpr int KK = 11; CALL; } break;     \
        case 12: { constexpr int KK = 12; CALL; } break;     \
        case 13: { constexpr int KK = 13; CALL; } break;     \
        case 14: { constexpr int KK = 14; CALL; } break;     \
        case 15: { constexpr int KK = 15; CALL; } break;     \
        case 16: { constexpr int KK = 16; CALL; } break;     \
        default: return NMF_EINVAL;                    \
    }

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct IpmLayout {
    size_t r, s, dx, dy, dr, ds, gx, gy, V, tX, tY, Lq, Linv, Rrow, Z, S, vec, vec2, XX, Dinv, spart, flags, part, fpart,
        sc, rhs0, dacc, Top, Hop, opart, Vex, kpart, total;
    int64_t vrows, kpart_cap;
    int64_t ldX, ldY, ldS;
    int P;
};

// Row splits of the Schur formation (split p of block b is b mod P).  Large
// problems (enough tile pairs to fill the chip many times) use one split.
// Otherwise 7: at 3000x500x5 the formation and split reduction took 544 us
// with 7 splits against 565 us with 8 (where each of the 8 XCDs would stream
// the Z rows of one split only), 578 with 6 and 569-582 with 12-16; the split
// count sets how evenly the blocks fill the chip's rounds of resident blocks,
// and that outweighs the L2 locality.
static int schur_splits(int64_t n, int64_t m, int K) {
    const int64_t T = (m + 15) / 16;
    const int64_t units = T * (T + 1) / 2 * schur_chunks(K);
    if (units >= 8192 || n < 8 * 32) return 1;
    return 7;
}

constexpr int OPS = 16;   // row splits of the operator's column pass

// Rows of the exact-Hessian factor V written out at a time (V holds n K rows
// of ldS entries): all of them up to 2 GiB, else slabs of that size.
static int64_t vex_rows(int64_t n, int K, int64_t ldS) {
    const int64_t nk = n * K;
    const int64_t cap = std::max<int64_t>(32, ((int64_t)2 << 30) / (ldS * 8));
    return std::min<int64_t>(std::min<int64_t>(nk, cap), 65535);
}

static IpmLayout ipm_layout(int64_t n, int64_t m_cap, int K) {
    IpmLayout L;
    L.ldX = (n + 63) / 64 * 64;
    L.ldY = (m_cap + 63) / 64 * 64;
    const int64_t N = m_cap * K;
    L.ldS = (N + 63) / 64 * 64;
    const int NL = K * (K + 1) / 2;
    const int64_t Tn = (n + XTILE - 1) / XTILE;
    // block records: rows + columns, then a second column-sized range
    const int64_t nblk = (n + NTHR - 1) / NTHR + 2 * ((m_cap + NTHR - 1) / NTHR) + 4;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off = al(off + bytes); return at; };
    const size_t vx = (size_t)K * L.ldX * 8, vy = (size_t)K * L.ldY * 8;
    L.r = take(vx); L.dx = take(vx); L.dr = take(vx); L.gx = take(vx); L.V = take(vx); L.tX = take(vx);
    L.s = take(vy); L.dy = take(vy); L.ds = take(vy); L.gy = take(vy); L.tY = take(vy);
    L.Lq = take((size_t)(NL + K) * L.ldX * 8);
    L.Linv = take((size_t)n * K * K * 8);
    L.Rrow = take((size_t)n * L.ldY * 8);
    L.Z = take((size_t)n * zpad(K) * L.ldY * 8);
    L.S = take((size_t)L.ldS * L.ldS * 8);
    L.vec = take((size_t)L.ldS * 8);
    L.vec2 = take((size_t)L.ldS * 8);
    L.XX = take((size_t)n * NL * 8);
    const int64_t NT = L.ldS / CB;
    L.Dinv = take((size_t)NT * CB * CB * 8);
    L.P = schur_splits(n, m_cap, K);
    const int64_t T16 = (m_cap + 15) / 16;
    L.spart = take(L.P > 1 ? (size_t)L.P * (T16 * (T16 + 1) / 2) * NL * 256 * 8 : 256);
    L.flags = take((size_t)3 * NT * sizeof(unsigned));
    L.part = take((size_t)nblk * PRS * 8);
    L.fpart = take((size_t)Tn * 64 * 8 * sizeof(double));   // Tn * Sx records of 8 (Sx <= 64)
    L.sc = take(sizeof(IpmScal));
    L.rhs0 = take((size_t)L.ldS * 8);
    L.dacc = take((size_t)L.ldS * 8);
    L.Top = take((size_t)n * L.ldY * 8);
    L.Hop = take((size_t)n * K * 8);
    L.opart = take((size_t)OPS * K * L.ldY * 8);
    L.vrows = vex_rows(n, K, L.ldS);
    L.Vex = take((size_t)L.vrows * L.ldS * 8);
    // partial tiles of the exact-Hessian rank update split over rows, sized
    // for the split count chosen at this capacity (fewer columns give fewer
    // tiles, whose chosen splits fit the same space)
    const int64_t T2 = (NT + 1) / 2, tiles = T2 * (T2 + 1) / 2;
    const int ns = tiles < 256 ? syrk_splits(tiles, INT64_MAX) : 1;
    L.kpart_cap = ns > 1 ? (int64_t)ns * tiles * 32 * 512 : 0;
    L.kpart = take(L.kpart_cap > 0 ? (size_t)L.kpart_cap * 8 : 256);
    L.total = off;
    return L;
}

size_t ipm_workspace_bytes(int64_t n, int64_t m_cap, int K) { return ipm_layout(n, m_cap, K).total + 256; }

nmf_status ipm_bind(IpmState &s, uint8_t *base, int64_t n, int64_t m_cap, int K) {
    const IpmLayout L = ipm_layout(n, m_cap, K);
    s.n = n; s.m_cap = m_cap; s.K = K; s.ldX = L.ldX; s.ldY = L.ldY; s.ldS = L.ldS;
    s.r = (double *)(base + L.r); s.s = (double *)(base + L.s);
    s.dx = (double *)(base + L.dx); s.dy = (double *)(base + L.dy);
    s.dr = (double *)(base + L.dr); s.ds = (double *)(base + L.ds);
    s.gx = (double *)(base + L.gx); s.gy = (double *)(base + L.gy);
    s.V = (double *)(base + L.V); s.tX = (double *)(base + L.tX); s.tY = (double *)(base + L.tY);
    s.Lq = (double *)(base + L.Lq); s.Z = (double *)(base + L.Z);
    s.Linv = (double *)(base + L.Linv); s.Rrow = (double *)(base + L.Rrow);
    s.S = (double *)(base + L.S); s.vec = (double *)(base + L.vec); s.vec2 = (double *)(base + L.vec2);
    s.XX = (double *)(base + L.XX);
    s.Dinv = (double *)(base + L.Dinv);
    s.spart = (double *)(base + L.spart);
    s.flags = (unsigned *)(base + L.flags);
    s.P = L.P;
    s.flags_ready = false;
    s.epoch = 0;
    s.part = (double *)(base + L.part); s.fpart = (double *)(base + L.fpart);
    s.sc = (IpmScal *)(base + L.sc);
    s.rhs0 = (double *)(base + L.rhs0);
    s.dacc = (double *)(base + L.dacc);
    s.Top = (double *)(base + L.Top);
    s.Hop = (double *)(base + L.Hop);
    s.opart = (double *)(base + L.opart);
    s.Vex = (double *)(base + L.Vex);
    s.vrows = L.vrows;
    s.kpart = L.kpart_cap > 0 ? (double *)(base + L.kpart) : nullptr;
    s.kpart_cap = L.kpart_cap;
    s.bound = true;
    return NMF_OK;
}

const char *ipm_last_error(const IpmState &s) { return s.err.c_str(); }

namespace {

struct Ctx {
    IpmState &s;
    const AnlsParams &p;
    const nmf_options &o;
    hipStream_t st;
    IpmArgs ia;
    int K;
};

#define HCK(call)                                             \
    do {                                                      \
        hipError_t _e = (call);                               \
        if (_e != hipSuccess) {                               \
            c.s.err = std::string(#call) + ": " + hipGetErrorString(_e); \
            return NMF_EDEVICE;                               \
        }                                                     \
    } while (0)

dim3 g1(int64_t count) { return dim3((unsigned)((count + NTHR - 1) / NTHR)); }

hipError_t finish(Ctx &c, const double *part, int stride, int nblk, int nval, unsigned minmask, double *out) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(NTHR), 0, c.st, part, stride, nblk, nval, minmask, out);
    return hipGetLastError();
}

// The k_finish reduction folded into the kernel that writes the records.
FinArgs fin(Ctx &c, const double *part, int stride, int nblk, int nval, unsigned minmask, double *out) {
    FinArgs f;
    f.part = part;
    f.out = out;
    f.cnt = &c.s.sc->fin_cnt;
    f.stride = stride;
    f.nblk = nblk;
    f.nval = nval;
    f.minmask = minmask;
    return f;
}

// The k_finish outputs, f and the failure words (the end of the scalar
// block) in one device-to-host transfer and one synchronisation.
// Through the context's pinned buffer when it has one (a direct DMA, no
// staging copy).
nmf_status read_tail(Ctx &c, IpmScal &h) {
    const size_t bytes = sizeof(IpmScal) - offsetof(IpmScal, out);
    IpmScal *dst = c.s.hsc ? c.s.hsc : &h;
    HCK(hipMemcpyAsync(dst->out, c.s.sc->out, bytes, hipMemcpyDeviceToHost, c.st));
    HCK(hipStreamSynchronize(c.st));
    if (dst != &h) memcpy(h.out, dst->out, bytes);
    return NMF_OK;
}

nmf_status read_out(Ctx &c, double *host, int nval) {
    HCK(hipMemcpyAsync(host, c.s.sc->out, sizeof(double) * nval, hipMemcpyDeviceToHost, c.st));
    HCK(hipStreamSynchronize(c.st));
    return NMF_OK;
}

// Gradients (residual form), f, G_X and G_Y at the current point.
hipError_t point_products(Ctx &c) {
    const AnlsParams &p = c.p;
    hipError_t e;
    IPM_K_SWITCH(c.K, hipLaunchKernelGGL(k_rstream_x<KK>, dim3(p.Tn, p.Sx), dim3(STHR), 0, c.st, p, p.Y,
                                          p.bx_part, c.s.fpart));
    hipLaunchKernelGGL(k_sum_splits, dim3(g1(p.n).x, (unsigned)(c.K)), dim3(NTHR), 0, c.st, p.bx_part, p.Sx, c.K, p.ldX, p.n, c.s.gx);
    if ((e = finish(c, c.s.fpart, 1, p.Tn * p.Sx, 1, 0u, &c.s.sc->f)) != hipSuccess) return e;
    IPM_K_SWITCH(c.K, hipLaunchKernelGGL(k_rstream_y<KK>, dim3(p.Tm, p.Sy), dim3(STHR), 0, c.st, p, p.X,
                                          p.by_part));
    hipLaunchKernelGGL(k_sum_splits, dim3(g1(p.m).x, (unsigned)(c.K)), dim3(NTHR), 0, c.st, p.by_part, p.Sy, c.K, p.ldY, p.m, c.s.gy);
    IPM_K_SWITCH(c.K, hipLaunchKernelGGL(k_outer<KK>, g1(p.n), dim3(NTHR), 0, c.st, p.X, p.X, p.ldX, p.n, c.s.part,
                                          fin(c, c.s.part, PRS, p.Bx, c.K * c.K, 0u, c.s.sc->GX)));
    IPM_K_SWITCH(c.K, hipLaunchKernelGGL(k_outer<KK>, g1(p.m), dim3(NTHR), 0, c.st, p.Y, p.Y, p.ldY, p.m, c.s.part,
                                          fin(c, c.s.part, PRS, p.By, c.K * c.K, 0u, c.s.sc->GY)));
    return hipGetLastError();
}

// KKT sums at the current point for barrier parameter mu; fills S1, C0, Cmu,
// E0, Emu and f.
nmf_status kkt_enqueue(Ctx &c, double mu, int slot) {
    const AnlsParams &p = c.p;
    IPM_KS(c.K, hipLaunchKernelGGL(k_kkt<KK>, dim3(p.Bx + p.By), dim3(NTHR), 0, c.st, p, c.ia, mu,
                                   fin(c, c.s.part, PRS, p.Bx + p.By, 4, 0u, c.s.sc->out + slot)));
    HCK(hipGetLastError());
    return NMF_OK;
}

// Reads the KKT sums (slot `slot` of the scalar block read back in hs).
nmf_status kkt_parse(Ctx &c, const IpmScal &hs, int slot) {
    if (hs.solve_fail) {
        c.s.err = "a block of a triangular solve waited too long for the tile before it";
        return NMF_EDEVICE;
    }
    const double *h = hs.out + slot;
    const double f = hs.f;
    c.s.S1 = h[0];
    c.s.SR = h[3];
    c.s.C0 = h[1];
    c.s.Cmu = h[2];
    c.s.f = 0.5 * f;
    c.s.E0 = fmax(sqrt(h[0]), sqrt(h[1]));
    c.s.Emu = fmax(sqrt(h[0]), sqrt(h[2]));
    return NMF_OK;
}

nmf_status kkt(Ctx &c, double mu) {
    nmf_status st = kkt_enqueue(c, mu, 0);
    if (st != NMF_OK) return st;
    IpmScal hs;
    st = read_tail(c, hs);
    if (st != NMF_OK) return st;
    return kkt_parse(c, hs, 0);
}

// Device time of the work enqueued between prof_begin and prof_end (a
// synchronising measurement, used only by nmf_ipm_profile).
void prof_begin(Ctx &c) {
    if (c.s.prof) (void)hipEventRecord(c.s.pev[0], c.st);
}
void prof_end(Ctx &c, int slot) {
    if (!c.s.prof) return;
    (void)hipEventRecord(c.s.pev[1], c.st);
    (void)hipEventSynchronize(c.s.pev[1]);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.s.pev[0], c.s.pev[1]) == hipSuccess) {
        c.s.prof_ms[slot] += ms;
        c.s.prof_n[slot] += 1;
    }
}

// Flag arrays of the two triangular solves (2 x NT; a third NT is spare): zeroed once,
// then every launch that hands over through them uses a fresh epoch.
nmf_status ensure_flags(Ctx &c) {
    if (c.s.flags_ready) return NMF_OK;
    HCK(launch_fill_u32(c.s.flags, 3 * (c.s.ldS / CB), 0u, c.st));
    // failure words are cleared by a fill kernel: no host memory, nothing
    // that waits for the stream
    HCK(launch_fill_u32((unsigned *)&c.s.sc->solve_fail, 1, 0u, c.st));
    HCK(launch_fill_u32(&c.s.sc->fin_cnt, 1, 0u, c.st));
    c.s.flags_ready = true;
    c.s.epoch = 0;
    return NMF_OK;
}

unsigned next_epoch(Ctx &c) {
    if (++c.s.epoch == 0) ++c.s.epoch;   // 0 is the cleared state
    return c.s.epoch;
}

// S = L L^T in place (lower triangle), with the inverse of every diagonal
// tile of L; Np = N rounded up to whole tiles, the padding is the identity.
nmf_status cholesky(Ctx &c, int64_t N) {
    const int64_t Np = (N + CB - 1) / CB * CB;
    HCK(launch_pad_identity(c.s.S, c.s.ldS, N, Np, c.st));
    CholArgs g;
    g.S = c.s.S;
    g.ldS = c.s.ldS;
    g.NT = (int)(Np / CB);
    g.Dinv = c.s.Dinv;
    g.fail = &c.s.sc->chol_fail;
    HCK(launch_cholesky(g, c.st));
    return NMF_OK;
}

// vec2 = S^-1 vec with the factor of cholesky(); vec is left as is.
nmf_status solve_S(Ctx &c, int64_t N) {
    HCK(ensure_flags(c) == NMF_OK ? hipSuccess : hipErrorUnknown);
    const int64_t Np = (N + CB - 1) / CB * CB;
    const int NT = (int)(Np / CB);
    const int64_t NTcap = c.s.ldS / CB;
    SolveArgs f;
    f.S = c.s.S;
    f.ldS = c.s.ldS;
    f.NT = NT;
    f.Dinv = c.s.Dinv;
    f.b = c.s.vec;
    f.y = c.s.vec2;
    f.flags = c.s.flags + NTcap;
    f.epoch = next_epoch(c);
    f.fail = &c.s.sc->solve_fail;
    SolveArgs bk = f;
    bk.b = nullptr;
    bk.flags = c.s.flags + 2 * NTcap;
    bk.epoch = next_epoch(c);
    HCK(launch_solve(f, bk, c.st));
    return NMF_OK;
}

struct Dir {
    bool ok;        // false: Cholesky of S failed
    double slope, a1, a2;
    bool formed = false;   // S was formed and factored for this direction (its failure flag is pending)
};

// Newton direction of eq. (12) at the current point with barrier parameter
// mu (0 for the predictor) and the Hessian eq. (26) (exact = false) or eq.
// (27) (exact = true), enqueued without synchronising.  Leaves dx, dy, dr, ds,
// the slope and step limits in out[OUT_DIR..] and, when S was factored, the
// factorisation flag; d.formed says whether it was.  The caller reads them in
// its own round trip.
nmf_status direction(Ctx &c, double mu, bool exact, double tau, Dir &d) {
    const AnlsParams &p = c.p;
    const int K = c.K;
    const int64_t N = p.m * K;
    const double rho = c.s.rho;
    // factors of Q1bar, V = Q1bar^-1 b1, X^T V
    IPM_KS(K, hipLaunchKernelGGL(k_factor<KK>, g1(p.n), dim3(NTHR), 0, c.st, p, c.ia, mu, rho));
    IPM_KS(K, hipLaunchKernelGGL(k_outer<KK>, g1(p.n), dim3(NTHR), 0, c.st, p.X, c.s.V, p.ldX, p.n, c.s.part,
                                 fin(c, c.s.part, PRS, p.Bx, K * K, 0u, c.s.sc->XtV)));
    const bool reuse = !exact && c.s.S_gn_valid;
    bool formed = false;
    if (!reuse) {
        HCK(launch_fill_u32((unsigned *)&c.s.sc->chol_fail, 1, 0u, c.st));
        IPM_KS(K, hipLaunchKernelGGL(k_zmat<KK>, dim3((unsigned)((p.n + ZRB - 1) / ZRB)), dim3(NTHR), 0, c.st,
                                           p, c.ia));
        const int64_t nt = (p.m + TJ - 1) / TJ;
        prof_begin(c);
        if (exact) {
            HCK(launch_linv(K, c.s.Lq, p.ldX, p.n, c.s.Linv, c.st));
            HCK(launch_residual_rows(K, p.M, p.ldM, p.X, p.ldX, p.Y, p.ldY, p.n, p.m, c.s.Rrow, c.st));
            SchurExArgs g;
            g.Z = c.s.Z;
            g.X = p.X;
            g.Linv = c.s.Linv;
            g.R = c.s.Rrow;
            g.n = p.n;
            g.m = p.m;
            g.ldX = p.ldX;
            g.ldY = p.ldY;
            g.NT = (int)((N + CB - 1) / CB);
            g.S = c.s.S;
            g.ldS = c.s.ldS;
            g.GX = c.s.sc->GX;
            g.s = c.s.s;
            g.Y = p.Y;
            g.rho = rho;
            HCK(launch_schur_exact_rows(K, g, c.s.Vex, c.s.ldS, c.s.vrows, c.s.mixed != 0, c.s.kpart, c.s.kpart_cap,
                                        c.st));
        } else {
            HCK(launch_xx(K, p.X, p.ldX, p.n, c.s.XX, c.st));
            SchurArgs g;
            g.Z = c.s.Z;
            g.XX = c.s.XX;
            g.n = p.n;
            g.m = p.m;
            g.ldY = p.ldY;
            g.npairs = (int)(nt * (nt + 1) / 2);
            g.P = c.s.P;
            g.rows_per_split = (p.n + g.P - 1) / g.P;
            g.part = c.s.spart;
            g.S = c.s.S;
            g.ldS = c.s.ldS;
            g.GX = c.s.sc->GX;
            g.s = c.s.s;
            g.Y = p.Y;
            g.rho = rho;
            HCK(launch_schur_gn(K, g, c.st));
        }
        prof_end(c, exact ? 1 : 0);
        prof_begin(c);
        nmf_status st = cholesky(c, N);
        if (st != NMF_OK) return st;
        prof_end(c, 2);
        // the factorisation's failure flag is read with the direction's
        // scalars (one host round trip less): a failed factor yields a
        // direction that is discarded
        formed = true;
        c.s.S_gn_valid = !exact;
    }
    if (exact) {
        IPM_KS(K, hipLaunchKernelGGL(k_rstream_y<KK>, dim3(p.Tm, p.Sy), dim3(STHR), 0, c.st, p, c.s.V,
                                           p.by_part));
        hipLaunchKernelGGL(k_sum_splits, dim3(g1(p.m).x, (unsigned)(K)), dim3(NTHR), 0, c.st, p.by_part, p.Sy, K, p.ldY, p.m, c.s.tY);
        IPM_KS(K, hipLaunchKernelGGL((k_rhs<KK, true>), g1(p.m), dim3(NTHR), 0, c.st, p, c.ia, mu));
    } else {
        IPM_KS(K, hipLaunchKernelGGL((k_rhs<KK, false>), g1(p.m), dim3(NTHR), 0, c.st, p, c.ia, mu));
    }
    prof_begin(c);
    nmf_status st = solve_S(c, N);
    if (st != NMF_OK) return st;
    if (exact && c.s.mixed) {
        // iterative refinement against the FP64 operator: d += S32^-1 (rhs - S d)
        const int64_t Np = (N + CB - 1) / CB * CB;
        HCK(hipMemcpyAsync(c.s.rhs0, c.s.vec, (size_t)Np * 8, hipMemcpyDeviceToDevice, c.st));
        HCK(hipMemcpyAsync(c.s.dacc, c.s.vec2, (size_t)Np * 8, hipMemcpyDeviceToDevice, c.st));
        OpArgs g;
        g.Z = c.s.Z;
        g.X = p.X;
        g.Linv = c.s.Linv;
        g.R = c.s.Rrow;
        g.n = p.n;
        g.m = p.m;
        g.ldX = p.ldX;
        g.ldY = p.ldY;
        g.v = c.s.dacc;
        g.T = c.s.Top;
        g.H = c.s.Hop;
        g.S = OPS;
        g.part = c.s.opart;
        g.GX = c.s.sc->GX;
        g.s = c.s.s;
        g.Y = p.Y;
        g.rho = rho;
        g.rhs = c.s.rhs0;
        g.res = c.s.vec;
        g.Np = Np;
        for (int it = 0; it < c.s.refine; ++it) {
            HCK(launch_schur_apply(K, true, g, c.st));
            st = solve_S(c, N);
            if (st != NMF_OK) return st;
            HCK(launch_axpy(c.s.dacc, c.s.vec2, Np, c.st));
        }
        HCK(hipMemcpyAsync(c.s.vec2, c.s.dacc, (size_t)Np * 8, hipMemcpyDeviceToDevice, c.st));
        HCK(hipMemcpyAsync(c.s.vec, c.s.rhs0, (size_t)Np * 8, hipMemcpyDeviceToDevice, c.st));
    }
    prof_end(c, 3);
    IPM_KS(K, hipLaunchKernelGGL(k_post_y<KK>, g1(p.m), dim3(NTHR), 0, c.st, p, c.ia, mu, tau, 0));
    IPM_KS(K, hipLaunchKernelGGL(k_outer<KK>, g1(p.m), dim3(NTHR), 0, c.st, c.s.dy, p.Y, p.ldY, p.m,
                                 c.s.part + (size_t)(p.By + p.Bx) * PRS,
                                 fin(c, c.s.part + (size_t)(p.By + p.Bx) * PRS, PRS, p.By, K * K, 0u, c.s.sc->T)));
    if (exact) {
        IPM_KS(K, hipLaunchKernelGGL(k_rstream_x<KK>, dim3(p.Tn, p.Sx), dim3(STHR), 0, c.st, p, c.s.dy,
                                           p.bx_part, (double *)nullptr));
        hipLaunchKernelGGL(k_sum_splits, dim3(g1(p.n).x, (unsigned)(K)), dim3(NTHR), 0, c.st, p.bx_part, p.Sx, K, p.ldX, p.n, c.s.tX);
        IPM_KS(K, hipLaunchKernelGGL((k_post_x<KK, true>), g1(p.n), dim3(NTHR), 0, c.st, p, c.ia, mu, tau,
                                     p.By, fin(c, c.s.part, PRS, p.By + p.Bx, 3, 0x6u, c.s.sc->out + OUT_DIR)));
    } else {
        IPM_KS(K, hipLaunchKernelGGL((k_post_x<KK, false>), g1(p.n), dim3(NTHR), 0, c.st, p, c.ia, mu, tau,
                                     p.By, fin(c, c.s.part, PRS, p.By + p.Bx, 3, 0x6u, c.s.sc->out + OUT_DIR)));
    }
    HCK(hipGetLastError());
    d.formed = formed;
    return NMF_OK;
}

// Enqueues the line search's quartic (k_ls_quartic) and its first batch of
// NTRIAL barrier trials from the direction's step limit (read on the device).
nmf_status probe_enqueue(Ctx &c) {
    const AnlsParams &p = c.p;
    double *lspart = c.s.fpart;   // reused: Tn*Sx records of 8
    IPM_KS(c.K, hipLaunchKernelGGL(k_ls_quartic<KK>, dim3(p.Tn, p.Sx), dim3(STHR), 0, c.st, p, c.ia, lspart));
    HCK(finish(c, lspart, 8, p.Tn * p.Sx, 6, 0u, c.s.sc->out + OUT_QUART));
    IPM_KS(c.K, hipLaunchKernelGGL(k_ls_barrier<KK>, dim3(p.Bx + p.By, NTRIAL / LS_TG), dim3(NTHR), 0, c.st, p, c.ia,
                                   (const double *)(c.s.sc->out + OUT_DIR + 1), 0.0,
                                   fin(c, c.s.part, PRS, p.Bx + p.By, NTRIAL, 0u, c.s.sc->out + OUT_BAR)));
    HCK(hipGetLastError());
    return NMF_OK;
}

// The direction's scalars, the quartic and the first barrier batch from the
// scalar block read back in hs.
void probe_parse(Ctx &c, Dir &d, const IpmScal &hs, double *q, double *bar) {
    const double *h = hs.out;
    for (int t = 0; t < 6; ++t) q[t] = h[OUT_QUART + t];
    for (int t = 0; t < NTRIAL; ++t) bar[t] = h[OUT_BAR + t];
    if (d.formed && hs.chol_fail) {
        c.s.S_gn_valid = false;
        d.ok = false;
        return;
    }
    d.ok = true;
    d.slope = h[OUT_DIR];
    d.a1 = h[OUT_DIR + 1] < 1.0 ? h[OUT_DIR + 1] : 1.0;
    d.a2 = h[OUT_DIR + 2] < 1.0 ? h[OUT_DIR + 2] : 1.0;
}

// The line-search inputs in one host round trip.
nmf_status probe(Ctx &c, Dir &d, double *q, double *bar) {
    nmf_status st = probe_enqueue(c);
    if (st != NMF_OK) return st;
    IpmScal hs;
    st = read_tail(c, hs);
    if (st != NMF_OK) return st;
    probe_parse(c, d, hs, q, bar);
    return NMF_OK;
}

// Armijo backtracking (eq. (13)) on the closed-form quartic q plus batched
// barrier sums; the first batch (bar) comes from probe().  Returns the
// accepted step in *al.
nmf_status line_search(Ctx &c, const Dir &d, double mu, const double *q, const double *bar0, double *al) {
#pragma clang fp contract(off)
    const AnlsParams &p = c.p;
    const int maxb = c.o.max_backtracks;
    for (int t0 = 0; t0 <= maxb; t0 += NTRIAL) {
        double barv[NTRIAL];
        const double *bar = bar0;
        if (t0 > 0) {
            const double abase = d.a1 / ldexp(1.0, t0);
            IPM_KS(c.K, hipLaunchKernelGGL(k_ls_barrier<KK>, dim3(p.Bx + p.By, NTRIAL / LS_TG), dim3(NTHR), 0, c.st, p,
                                           c.ia, (const double *)nullptr, abase,
                                           fin(c, c.s.part, PRS, p.Bx + p.By, NTRIAL, 0u, c.s.sc->out)));
            HCK(hipGetLastError());
            nmf_status st = read_out(c, barv, NTRIAL);
            if (st != NMF_OK) return st;
            bar = barv;
        }
        for (int t = 0; t < NTRIAL && t0 + t <= maxb; ++t) {
            const double a = d.a1 / ldexp(1.0, t0 + t);
            const double dq = 0.5 * (2.0 * a * q[1] + a * a * (q[2] + 2.0 * q[3]) + 2.0 * a * a * a * q[4] +
                                     a * a * a * a * q[5]);
            const double dphi = dq - mu * bar[t];
            if (dphi <= c.o.eta * a * d.slope) {
                c.s.backtracks += t0 + t;
                *al = a;
                return NMF_OK;
            }
        }
    }
    c.s.backtracks += maxb;
    c.s.cap_hits += 1;
    *al = d.a1 / ldexp(1.0, maxb);
    return NMF_OK;
}

// The update (step a1, a2, or the device's choice in sel), the products at
// the new point and its KKT sums into slot `slot`, without synchronising.
nmf_status update_enqueue(Ctx &c, double a1, double a2, const double *sel, int slot) {
    const AnlsParams &p = c.p;
    const int64_t e = p.n > p.m ? p.n : p.m;
    IPM_KS(c.K, hipLaunchKernelGGL(k_update<KK>, g1(e), dim3(NTHR), 0, c.st, p, c.ia, a1, a2, sel));
    HCK(point_products(c));
    return kkt_enqueue(c, c.s.mu, slot);
}

nmf_status update_point(Ctx &c, double a1, double a2) {
    nmf_status st = update_enqueue(c, a1, a2, nullptr, 0);
    if (st != NMF_OK) return st;
    c.s.S_gn_valid = false;
    IpmScal hs;
    st = read_tail(c, hs);
    if (st != NMF_OK) return st;
    return kkt_parse(c, hs, 0);
}

// One inner iteration of Alg. 3 (direction with the flag rule, step rules,
// Armijo search, update).
nmf_status inner_iteration(Ctx &c) {
    IpmState &s = c.s;
    const double mu = s.mu;
    Dir d;
    d.ok = false;
    bool have = false;
    nmf_status st;
    double q[6], bar[NTRIAL];
    if (s.flag == 1 && c.o.exact_hessian_switch) {
        st = direction(c, mu, true, c.o.tau, d);
        if (st != NMF_OK) return st;
        st = probe(c, d, q, bar);
        if (st != NMF_OK) return st;
        if (d.ok && d.slope < 0.0) {
            have = true;
            s.exact_steps += 1;
        } else {
            s.flag = 0;
            s.fallbacks += 1;
        }
    }
    if (!have) {
        d = Dir();
        d.ok = false;
        st = direction(c, mu, false, c.o.tau, d);
        if (st != NMF_OK) return st;
        // The line-search inputs, the first Armijo batch, the update and the
        // KKT sums of the new point are enqueued together and read back in
        // one round trip; when no trial of the first batch is accepted the
        // device leaves the point as it is and the host continues the search.
        st = probe_enqueue(c);
        if (st != NMF_OK) return st;
        hipLaunchKernelGGL(k_armijo, dim3(1), dim3(64), 0, c.st, s.sc, mu, c.o.eta, c.o.max_backtracks,
                           d.formed ? 1 : 0);
        HCK(hipGetLastError());
        st = update_enqueue(c, 0.0, 0.0, s.sc->out + OUT_SEL, OUT_KKT);
        if (st != NMF_OK) return st;
        IpmScal hs;
        st = read_tail(c, hs);
        if (st != NMF_OK) return st;
        probe_parse(c, d, hs, q, bar);
        if (!d.ok) {
            s.err = "Cholesky factorisation of the Gauss-Newton Schur matrix failed";
            return NMF_ESINGULAR;
        }
        const double *sel = hs.out + OUT_SEL;
        if (sel[0] != 0.0) {
            s.backtracks += (int)sel[3];
            s.iters += 1;
            s.at_mu += 1;
            s.S_gn_valid = false;
            return kkt_parse(c, hs, OUT_KKT);
        }
        if (hs.solve_fail) {
            s.err = "a block of a triangular solve waited too long for the tile before it";
            return NMF_EDEVICE;
        }
    }
    double al = 0.0;
    st = line_search(c, d, mu, q, bar, &al);
    if (st != NMF_OK) return st;
    s.iters += 1;
    s.at_mu += 1;
    return update_point(c, al, d.a2);
}

// Predictor probe and the mu update of Alg. 3 (eq. (8), (9)).
nmf_status mu_update(Ctx &c) {
    IpmState &s = c.s;
    const AnlsParams &p = c.p;
    Dir d;
    d.ok = false;
    // the predictor direction and its complementarity sum, read back together
    nmf_status st = direction(c, 0.0, false, 1.0, d);
    if (st != NMF_OK) return st;
    IPM_KS(c.K, hipLaunchKernelGGL(k_muaff<KK>, dim3(p.Bx + p.By), dim3(NTHR), 0, c.st, p, c.ia, 0.0, 0.0,
                                   (const double *)(s.sc->out + OUT_DIR + 1),
                                   fin(c, s.part, PRS, p.Bx + p.By, 1, 0u, s.sc->out + OUT_AFF)));
    HCK(hipGetLastError());
    IpmScal hs;
    st = read_tail(c, hs);
    if (st != NMF_OK) return st;
    if (d.formed && hs.chol_fail) {
        s.S_gn_valid = false;
        s.err = "Cholesky factorisation of the predictor Schur matrix failed";
        return NMF_ESINGULAR;
    }
    const double Nn = (double)(p.n + p.m) * c.K;
    const double avg = s.SR / Nn;   // current average complementarity
    const double mu_aff = hs.out[OUT_AFF] / Nn;
    // mu_aff is a complementarity of points in the closed orthant, so it is
    // >= 0; the step to the boundary (tau = 1) can leave a rounding residue
    // below 0, which must not turn sigma (and mu) negative.
    double r = mu_aff > 0.0 ? mu_aff / avg : 0.0;
    double sigma = r * r * r;
    if (sigma > 0.99) sigma = 0.99;
    s.sigma = sigma;
    s.mu = sigma * avg;
    s.flag = (sigma <= c.o.sigma_c) ? 1 : 0;
    return kkt(c, s.mu);
}

}  // namespace

nmf_status ipm_transition(IpmState &s, const AnlsParams &p, const nmf_options &o, hipStream_t st) {
    if (!s.bound) { s.err = "no stage-2 workspace"; return NMF_ESTATE; }
    Ctx c{s, p, o, st, args_of(s), s.K};
    // the hand-over flags and the solve-failure word start cleared (the
    // workspace arrives uninitialised)
    s.flags_ready = false;
    if (ensure_flags(c) != NMF_OK) return NMF_EDEVICE;
    // rho0 = 1e-6 max(x, y) on the stage-1 point, eq. (22)
    IPM_KS(c.K, hipLaunchKernelGGL(k_maxes<KK>, dim3(p.Bx + p.By), dim3(NTHR), 0, st, p, c.ia, 0));
    HCK(finish(c, s.part, PRS, p.Bx + p.By, 2, 0x3u, s.sc->out));
    double mx[2];
    nmf_status r = read_out(c, mx, 2);
    if (r != NMF_OK) return r;
    const double vmax = fmax(-mx[0], -mx[1]);
    const double rho0 = o.rho0_factor * vmax;
    IPM_KS(c.K, hipLaunchKernelGGL(k_clamp<KK>, g1(p.n > p.m ? p.n : p.m), dim3(NTHR), 0, st, p, rho0));
    HCK(point_products(c));
    // r = max |graX| e, s = max |graY| e at the clamped point, eq. (23)
    IPM_KS(c.K, hipLaunchKernelGGL(k_maxes<KK>, dim3(p.Bx + p.By), dim3(NTHR), 0, st, p, c.ia, 1));
    HCK(finish(c, s.part, PRS, p.Bx + p.By, 2, 0x3u, s.sc->out));
    r = read_out(c, mx, 2);
    if (r != NMF_OK) return r;
    const double rv = fmax(-mx[0], o.eps_tol), sv = fmax(-mx[1], o.eps_tol);
    IPM_KS(c.K, hipLaunchKernelGGL(k_fill_duals<KK>, dim3(p.Bx + p.By), dim3(NTHR), 0, st, p, c.ia, rv, sv));
    HCK(finish(c, s.part, PRS, p.Bx + p.By, 2, 0u, s.sc->out));
    double sums[2];
    r = read_out(c, sums, 2);
    if (r != NMF_OK) return r;
    const double Nn = (double)(p.n + p.m) * c.K;
    s.mu = (rv * sums[0] + sv * sums[1]) / Nn;   // eq. (24)
    s.rho = o.rho;                               // eq. (25)
    s.flag = 0;
    s.in_inner = false;
    s.S_gn_valid = false;
    s.at_mu = 0;
    s.iters = s.outer = s.backtracks = s.exact_steps = s.fallbacks = s.cap_hits = 0;
    s.sigma = 0.0;
    return kkt(c, s.mu);
}

nmf_status ipm_iterate(IpmState &s, const AnlsParams &p, const nmf_options &o, int iters, hipStream_t st) {
    Ctx c{s, p, o, st, args_of(s), s.K};
    int budget = iters;
    for (;;) {
        if (!s.in_inner) {
            if (s.E0 <= o.eps_tol) return NMF_CONVERGED;
            if (s.iters >= o.max_ipm_iters || s.outer >= o.max_ipm_iters) return NMF_ENOTCONV;
            s.outer += 1;
            s.eps_mu = s.mu;
            s.at_mu = 0;
            s.in_inner = true;
        }
        if (s.Emu > s.eps_mu && s.E0 > o.eps_tol && s.iters < o.max_ipm_iters && s.at_mu < o.inner_cap) {
            if (budget <= 0) return NMF_OK;
            nmf_status r = inner_iteration(c);
            if (r != NMF_OK) return r;
            --budget;
            continue;
        }
        s.in_inner = false;
        if (s.E0 <= o.eps_tol) return NMF_CONVERGED;
        if (s.iters >= o.max_ipm_iters) return NMF_ENOTCONV;
        nmf_status r = mu_update(c);
        if (r != NMF_OK) return r;
    }
}

nmf_status ipm_report(IpmState &s, nmf_report *r, double ms1, double ms2) {
    r->stage = 2;
    r->f = s.f;
    r->E0 = s.E0;
    r->Emu = s.Emu;
    r->mu = s.mu;
    r->sigma = s.sigma;
    r->flag = s.flag;
    r->ipm_iters = s.iters;
    r->ipm_outer = s.outer;
    r->backtracks = s.backtracks;
    r->exact_steps = s.exact_steps;
    r->fallbacks = s.fallbacks;
    r->ms_stage1 = ms1;
    r->ms_stage2 = ms2;
    return NMF_OK;
}

nmf_status ipm_export(IpmState &s, const AnlsParams &p, hipStream_t st) {
    if (!s.bound) return NMF_OK;
    const int64_t e = p.n > p.m ? p.n : p.m;
    switch (s.K) {
#define MK(KK) case KK: hipLaunchKernelGGL(k_masks<KK>, dim3((unsigned)((e + NTHR - 1) / NTHR)), dim3(NTHR), 0, st, p); break;
        MK(1) MK(2) MK(3) MK(4) MK(5) MK(6) MK(7) MK(8) MK(9) MK(10) MK(11) MK(12) MK(13) MK(14) MK(15) MK(16)
#undef MK
        default: return NMF_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

nmf_status ipm_get_duals(IpmState &s, const AnlsParams &p, double *R, double *S, hipStream_t st) {
    if (!s.bound) return NMF_ESTATE;
    const int64_t e = p.n > p.m ? p.n : p.m;
    IpmArgs ia = args_of(s);
    double *stR = s.tX, *stS = s.tY;
    switch (s.K) {
#define MK(KK) case KK: hipLaunchKernelGGL(k_duals_out<KK>, dim3((unsigned)((e + NTHR - 1) / NTHR)), dim3(NTHR), 0, st, p, ia, R ? stR : nullptr, S ? stS : nullptr); break;
        MK(1) MK(2) MK(3) MK(4) MK(5) MK(6) MK(7) MK(8) MK(9) MK(10) MK(11) MK(12) MK(13) MK(14) MK(15) MK(16)
#undef MK
        default: return NMF_EINVAL;
    }
    if (R && hipMemcpyAsync(R, stR, (size_t)p.n * s.K * 8, hipMemcpyDefault, st) != hipSuccess) return NMF_EDEVICE;
    if (S && hipMemcpyAsync(S, stS, (size_t)p.m * s.K * 8, hipMemcpyDefault, st) != hipSuccess) return NMF_EDEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

}  // namespace nmfk
