// Stage 1 of the two-stage NMF: one ANLS sweep (Alg. 1) is four kernels.
//
//   k_xstream  B_X = M Y^T in split partials.  Grid (Tn tiles of 64 rows) x
//              (Sx column splits); 8 waves per block, each wave a slice of
//              the split's columns, eight 512-byte loads of M in flight per
//              wave; Y for the split is staged in LDS.
//   k_xnnls    one thread per row (one wave per block up to k = 8): sums the Sx
//              partials in order, reduces G_Y = Y Y^T from the records of the
//              last Y-half,
//              measures the KKT parts of E(.;0) at the old point (r =
//              max(graX, 0), Sec. V-A) and solves eq. (2) with C = Y^T by the
//              warm-started active-set method.  Each wave leaves its own
//              record of statistics and of the new G_X = X^T X (no block
//              barrier waits for a slower wave).
//   k_ystream  B_Y = X^T M in split partials.  Grid (Tm tiles of J = 64/K
//              columns) x (Sy row splits); every lane accumulates J*K dot
//              products and a wave transpose-reduce leaves one sum per lane.
//   k_ynnls    one thread per column (blocks as k_xnnls): eq. (2) with C = X;
//              a record of the new G_Y per wave; the last block applies the
//              stop rule of Sec. IV.
//
// All hand-overs between blocks cross a kernel boundary, except the sweep
// summary in k_ynnls.  Every sum runs in a fixed order,
// so results are bitwise reproducible.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/nmf.h"
#include "device_util.h"
#include "nmf_internal.h"
#include "nnls_lh.h"

namespace nmfk {

// ---------------------------------------------------------------- X-half
// Element (i, j) of M in the arithmetic type of precision P: FP64 from M,
// FP32 from the 4-byte copy, or the sum of its BF16 high and low parts.
template <int P>
struct MElem;
template <>
struct MElem<NMF_GRAM_FP64> {
    using T = double;
    static __device__ __forceinline__ double load(const AnlsParams &p, int64_t off) { return p.M[off]; }
    // elements off and off + 1 in one 16-byte load (off even)
    static __device__ __forceinline__ void load2(const AnlsParams &p, int64_t off, double &a, double &b) {
        const double2 v = *reinterpret_cast<const double2 *>(p.M + off);
        a = v.x;
        b = v.y;
    }
};
template <>
struct MElem<NMF_GRAM_FP32> {
    using T = float;
    static __device__ __forceinline__ float load(const AnlsParams &p, int64_t off) {
        return __uint_as_float(p.Mlo[off]);
    }
    static __device__ __forceinline__ void load2(const AnlsParams &p, int64_t off, float &a, float &b) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p.Mlo + off);
        a = __uint_as_float(u.x);
        b = __uint_as_float(u.y);
    }
};
template <>
struct MElem<NMF_GRAM_BF16X2> {
    using T = float;
    static __device__ __forceinline__ float load(const AnlsParams &p, int64_t off) {
        const uint32_t u = p.Mlo[off];
        return __uint_as_float(u & 0xFFFF0000u) + __uint_as_float(u << 16);
    }
    static __device__ __forceinline__ void load2(const AnlsParams &p, int64_t off, float &a, float &b) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p.Mlo + off);
        a = __uint_as_float(u.x & 0xFFFF0000u) + __uint_as_float(u.x << 16);
        b = __uint_as_float(u.y & 0xFFFF0000u) + __uint_as_float(u.y << 16);
    }
};

// Lane `src`'s value of v in every lane (one pivot or column entry of a
// lane-per-row factorisation).
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------- grouped first solves
// Passive-set grouping (the grouping of right-hand sides that share a passive
// set, cited in Sec. II): the problems of one half whose warm-start passive
// set P is the same share one factorisation of G_PP.  Per half and sweep,
// every problem marks its set (k_gmark), one block numbers the distinct sets
// (k_gnumber) and one wave per set forms (G_PP)^-1 (k_ginverse).  A problem
// then first tries z = (G_PP)^-1 b, the first solve of the warm-started
// Lawson-Hanson loop, and keeps it when z is positive on P and the dual
// vector passes the loop's optimality test; otherwise it runs the loop as
// before, from the same start.  The minimiser is the loop's (it is unique),
// up to the rounding of the solve.
template <int K>
__device__ __forceinline__ bool grouped_try(const AnlsParams &p, const double *G, double gmax, const double (&b)[K],
                                            const double (&x0)[K], uint32_t old_mask, double (&xn)[K]) {
    uint32_t barred = 0, P = 0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        if (!(G[a * K + a] > 1e-14 * gmax)) barred |= 1u << a;
        else if (x0[a] > 0.0) P |= 1u << a;
    }
    if (P != old_mask) return false;
    const int slot = p.gslot[P];
    if (slot < 0) return false;
    const double *T = p.gtab + (int64_t)slot * (K * K);
    double z[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c) v = fma(T[a * K + c], b[c], v);
        z[a] = ((P >> a) & 1u) ? v : 0.0;
    }
    bool feas = true;
#pragma unroll
    for (int a = 0; a < K; ++a)
        if (((P >> a) & 1u) && !(z[a] > 0.0)) feas = false;
    if (!feas) return false;
    // the optimality test of the loop, at x = z
    double tol = 0.0, wj = 0.0;
    int j = -1;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double v = b[a], s = fabs(b[a]);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            v -= G[a * K + c] * z[c];
            s += fabs(G[a * K + c]) * z[c];
        }
        tol = s > tol ? s : tol;
        if (!(((P | barred) >> a) & 1u)) {
            if (j < 0 || v > wj) { j = a; wj = v; }
        }
    }
    tol *= 10.0 * K * 2.220446049250313e-16;
    if (j >= 0 && wj > tol) return false;
#pragma unroll
    for (int a = 0; a < K; ++a) xn[a] = z[a];
    return true;
}

// The warm-started solve of one problem, grouped first when the half has a
// table this sweep.
template <int K>
__device__ __forceinline__ LhResult solve_warm(const AnlsParams &p, const double *G, double gmax,
                                               const double (&b)[K], uint32_t old_mask, double (&xn)[K]) {
    if (p.grouped) {
        double x0[K];
#pragma unroll
        for (int a = 0; a < K; ++a) x0[a] = xn[a];
        if (grouped_try<K>(p, G, gmax, b, x0, old_mask, xn)) {
            LhResult r;
            r.P = old_mask;
            r.solves = 1;
            r.status = 0;
            return r;
        }
    }
    return lh_warm<K>(G, gmax, b, xn);
}

// Row i of the X-half: the gradient statistics at the previous row x (E(.;0)
// parts), and in mode 0 the warm-started solve, stored to X and the mask.
// b is row i of B_X = M Y^T, G is G_Y in LDS.  xn receives the new row (zeros
// in mode 1).
template <int K>
__device__ __forceinline__ void x_row(const AnlsParams &p, const double *G, int64_t i, const double (&x)[K],
                                      const double (&b)[K], uint32_t old_mask, double (&st)[NST],
                                      double (&xn)[K]) {
    double gmax = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a) gmax = G[a * K + a] > gmax ? G[a * K + a] : gmax;
    // graX at the old point: (X Y Y^T - M Y^T)_i
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double g = -b[a];
#pragma unroll
        for (int c = 0; c < K; ++c) g = fma(G[a * K + c], x[c], g);
        if (g < 0.0) st[ST_EG2] += g * g;
        else st[ST_EC2] += (g * x[a]) * (g * x[a]);
    }
    if (p.mode == 0) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            xn[a] = x[a];
            st[ST_NORM2] += x[a] * x[a];
        }
        const LhResult r = solve_warm<K>(p, G, gmax, b, old_mask, xn);
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const double d = xn[a] - x[a];
            st[ST_STEP2] += d * d;
            p.X[(int64_t)a * p.ldX + i] = xn[a];
        }
        p.xmask[i] = r.P;
        st[ST_SOLVES] = r.solves;
        st[ST_FAILS] = r.status != 0 ? 1.0 : 0.0;
        st[ST_CHANGES] = r.P != old_mask ? 1.0 : 0.0;
    }
}

// Column j of the Y-half: warm-started solve from the previous column y,
// stored to Y and the mask, then the gradient statistics at the new column.
// b is column j of B_Y = X^T M, G is G_X in LDS.
template <int K>
__device__ __forceinline__ void y_col(const AnlsParams &p, const double *G, int64_t j, const double (&y)[K],
                                      const double (&b)[K], uint32_t old_mask, double (&st)[NST],
                                      double (&yn)[K]) {
    double gmax = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a) gmax = G[a * K + a] > gmax ? G[a * K + a] : gmax;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        yn[a] = y[a];
        st[ST_NORM2] += y[a] * y[a];
    }
    const LhResult r = solve_warm<K>(p, G, gmax, b, old_mask, yn);
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const double d = yn[a] - y[a];
        st[ST_STEP2] += d * d;
        p.Y[(int64_t)a * p.ldY + j] = yn[a];
    }
    p.ymask[j] = r.P;
    // graY at the new point: (X^T X Y - X^T M)_j, the Y part of E(.;0)
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double g = -b[a];
#pragma unroll
        for (int c = 0; c < K; ++c) g = fma(G[a * K + c], yn[c], g);
        if (g < 0.0) st[ST_EG2] += g * g;
        else st[ST_EC2] += (g * yn[a]) * (g * yn[a]);
    }
    st[ST_SOLVES] = r.solves;
    st[ST_FAILS] = r.status != 0 ? 1.0 : 0.0;
    st[ST_CHANGES] = r.P != old_mask ? 1.0 : 0.0;
}

// One wave's record: the sums over its 64 lanes of the statistics and of the
// products xn_a xn_c (a >= c); lane q writes value q of each 64-value pass
// (statistics to stat_out, the Gram matrix in both triangles to gram_out
// unless it is null).  Called by all 64 lanes of the wave.
// (a, c), a >= c, of entry idx of the packed lower triangle (row by row).
__host__ __device__ constexpr int tri_row(int idx) {
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= idx) ++a;
    return a;
}
__host__ __device__ constexpr int tri_col(int idx) { return idx - tri_row(idx) * (tri_row(idx) + 1) / 2; }

template <int K>
__device__ __forceinline__ void wave_stats_and_gram(const double (&st)[NST], const double (&xn)[K],
                                                    double *stat_out, double *gram_out) {
    constexpr int NG = K * (K + 1) / 2;
    constexpr int V = NG + NST;
    constexpr int NPASS = (V + YVALS - 1) / YVALS;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        constexpr int W = V <= 32 ? 32 : YVALS;
        double v[W];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int idx = pass * YVALS + q;
            if (idx < NG) v[q] = xn[tri_row(idx)] * xn[tri_col(idx)];
            else if (idx < V) v[q] = st[idx - NG];
            else v[q] = 0.0;
        }
        double sum;
        if constexpr (W == 32) sum = wave_transpose_reduce32(v, lane);
        else sum = wave_transpose_reduce(v, lane);
        const int idx = pass * YVALS + lane;
        if (idx < V) {
            if (idx >= NG) {
                stat_out[idx - NG] = sum;
            } else if (gram_out) {
                const int a = tri_row(idx), c = tri_col(idx);
                gram_out[a * K + c] = sum;
                gram_out[c * K + a] = sum;
            }
        }
    }
}

// The stage-1 stop flag of a sweep kernel (mode 0 only).  It is read with a
// vector load issued before the kernel's other loads: waiting for a scalar
// load would also wait for every kernel argument still in flight, and the
// flag would then cost a memory round trip of its own before any data moves.
__device__ __forceinline__ bool sweep_stopped(const AnlsParams &p) {
    const int conv = __hip_atomic_load(&p.st->converged, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (p.mode == 0) & (conv != 0);
}

// End of a sweep, in the block that finished last: the X and Y statistics
// records, the E(.;0) parts and the stop rule of Sec. IV (mode 0), or only the
// Y part for appended columns (mode 2).  All threads call it; scr holds
// blockDim doubles of LDS.
__device__ __forceinline__ void sweep_summary(const AnlsParams &p, double *scr) {
    __shared__ double sx[NST], sy[NST];
    DevStatus *s = p.st;
    // the status fields and both record sets are loaded together: the first
    // half of the block sums the X records, the second half the Y records
    double ey_g2 = 0.0, ey_c2 = 0.0, solves = 0.0, fails = 0.0, changes = 0.0, eps = 0.0;
    long long sweeps = 0, max_sweeps = 0;
    if (threadIdx.x == 0) {
        ey_g2 = s->ey_g2;
        ey_c2 = s->ey_c2;
        solves = s->solves;
        fails = s->fails;
        changes = s->changes;
        eps = s->eps_stol;
        sweeps = s->sweeps;
        max_sweeps = s->max_sweeps;
    }
    const int half = (int)blockDim.x / 2;
    const bool yside = (int)threadIdx.x >= half;
    const int tid = yside ? (int)threadIdx.x - half : (int)threadIdx.x;
    const double acc = yside ? records_partial(p.ystat, p.Ry, NST, tid, half)
                             : records_partial(p.xstat, p.Rx, NST, tid, half);
    scr[threadIdx.x] = acc;
    __syncthreads();
    if (tid < NST) {
        const int G = half / NST;
        double v = 0.0;
        for (int gg = 0; gg < G; ++gg) v += scr[(yside ? half : 0) + gg * NST + tid];
        (yside ? sy : sx)[tid] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0 && p.mode == 2) {
        // appended columns solved: Y part of E, counters; no sweep, no stop test
        s->ey_g2 = sy[ST_EG2];
        s->ey_c2 = sy[ST_EC2];
        s->E_cur = -1.0;
        s->solves = solves + sy[ST_SOLVES];
        s->fails = fails + sy[ST_FAILS];
        s->changes = changes + sy[ST_CHANGES];
    } else if (threadIdx.x == 0) {
        const double step2 = sx[ST_STEP2] + sy[ST_STEP2];
        const double norm2 = sx[ST_NORM2] + sy[ST_NORM2];
        s->step2 = step2;
        s->norm2 = norm2;
        s->ex_g2 = sx[ST_EG2];
        s->ex_c2 = sx[ST_EC2];
        if (ey_g2 >= 0.0) {
            const double eg = sqrt(sx[ST_EG2] + ey_g2);
            const double ec = sqrt(sx[ST_EC2] + ey_c2);
            s->E_prev = eg > ec ? eg : ec;
        }
        s->ey_g2_prev = ey_g2;
        s->ey_c2_prev = ey_c2;
        s->ey_g2 = sy[ST_EG2];
        s->ey_c2 = sy[ST_EC2];
        s->E_cur = -1.0;
        s->solves = solves + (sx[ST_SOLVES] + sy[ST_SOLVES]);
        s->fails = fails + (sx[ST_FAILS] + sy[ST_FAILS]);
        s->changes = changes + (sx[ST_CHANGES] + sy[ST_CHANGES]);
        s->sweeps = sweeps + 1;
        if (sqrt(step2) <= eps * (1.0 + sqrt(norm2)) || sweeps + 1 >= max_sweeps) s->converged = 1;
    }
}

// LDS of the X stream: a chunk of Y while streaming, then the wave sums.
template <int K>
constexpr int xstream_lds() {
    return (XCHUNK * K > SWAVES * K * XTILE) ? XCHUNK * K : SWAVES * K * XTILE;
}

// Streams the columns [j0, j1) of the tile's 64 rows of M against Y and
// leaves each wave's partial sums of B_X in lds[(w * K + a) * XTILE + lane]
// (ends with a barrier).  The first chunk of Y and the first eight columns of
// each wave go out together with the caller's stop flag (a scalar load); with
// `stop` set the block returns false before touching LDS.  Every thread of the
// block calls it.
template <int K, int P>
__device__ __forceinline__ bool xstream_sums(const AnlsParams &p, int tile, int64_t j0, int64_t j1, double *lds,
                                             bool stop) {
    using T = typename MElem<P>::T;
    constexpr int NL = 8;   // loads in flight per lane
    constexpr int YPER = (XCHUNK * K + STHR - 1) / STHR;
    T *ys = reinterpret_cast<T *>(lds);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)tile * XTILE + lane;
    const bool row_ok = i < p.n;
    // lanes past the last row stream row n - 1; their sums are never used
    const int64_t ic = row_ok ? i : p.n - 1;

    T acc[K];
#pragma unroll
    for (int a = 0; a < K; ++a) acc[a] = T(0);
    for (int64_t c0 = j0; c0 < j1; c0 += XCHUNK) {
        const int nc = (int)min((int64_t)XCHUNK, j1 - c0);
        const int64_t base = c0 * p.ldM + ic;
        // all first loads of the chunk are issued without a branch between
        // them (indices clamped into the chunk; surplus values are not used)
        T yv[YPER], mv[NL];
#pragma unroll
        for (int u = 0; u < YPER; ++u) {
            const int q = min((int)threadIdx.x + u * STHR, nc * K - 1);
            const int jj = q / K, a = q - jj * K;
            yv[u] = (T)p.Y[(int64_t)a * p.ldY + c0 + jj];
        }
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int jj = min(w + t * SWAVES, nc - 1);
            mv[t] = MElem<P>::load(p, base + (int64_t)jj * p.ldM);
        }
        if (c0 == j0 && stop) return false;
        __syncthreads();   // the previous chunk's reads of ys are done
#pragma unroll
        for (int u = 0; u < YPER; ++u) {
            const int q = (int)threadIdx.x + u * STHR;
            if (q < nc * K) ys[q] = yv[u];
        }
        __syncthreads();
        for (int jb = w; jb < nc; jb += NL * SWAVES) {
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                const int jj = jb + t * SWAVES;
                if (jj < nc) {
#pragma unroll
                    for (int a = 0; a < K; ++a) acc[a] = fma(mv[t], ys[jj * K + a], acc[a]);
                }
            }
            const int jn = jb + NL * SWAVES;
            if (jn < nc) {
#pragma unroll
                for (int t = 0; t < NL; ++t) {
                    const int jj = min(jn + t * SWAVES, nc - 1);
                    mv[t] = MElem<P>::load(p, base + (int64_t)jj * p.ldM);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < K; ++a) lds[(w * K + a) * XTILE + lane] = (double)acc[a];
    __syncthreads();
    return true;
}

// X stream, one column split: partial sums of B_X for the split.
template <int K, int P>
__device__ __forceinline__ void xstream_body(const AnlsParams &p, int tile, int split, double *lds) {
    const bool stop = sweep_stopped(p);
    const int64_t j0 = (int64_t)split * p.xcols;
    const int64_t j1 = min(j0 + (int64_t)p.xcols, p.m);
    if (!xstream_sums<K, P>(p, tile, j0, j1, lds, stop)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)tile * XTILE + lane;
    if (w == 0 && i < p.n) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double v = lds[(0 * K + a) * XTILE + lane];
#pragma unroll
            for (int ww = 1; ww < SWAVES; ++ww) v += lds[(ww * K + a) * XTILE + lane];
            p.bx_part[((int64_t)split * K + a) * p.ldX + i] = v;
        }
    }
}

// Splits of the B partials summed per row (column), in split order; SB splits
// (SB * K loads) are in flight at a time and splits past S read as zero.
template <int K>
constexpr int partial_batch() {
    return (48 / K) < 1 ? 1 : ((48 / K) > 16 ? 16 : 48 / K);
}
template <int K>
__device__ __forceinline__ void sum_split_partials(const double *part, int64_t ld, int64_t i, int S,
                                                   double (&b)[K]) {
    constexpr int SB = partial_batch<K>();
    for (int s0 = 0; s0 < S; s0 += SB) {
        double t[SB][K];
        // every load is issued (splits past S re-read split S - 1) and the
        // surplus ones are dropped afterwards: no branch between the loads
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int su = s0 + u < S ? s0 + u : S - 1;
#pragma unroll
            for (int a = 0; a < K; ++a) t[u][a] = part[((int64_t)su * K + a) * ld + i];
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
#pragma unroll
            for (int a = 0; a < K; ++a) b[a] += (s0 + u < S) ? t[u][a] : 0.0;
        }
    }
}

// Sum over the S splits of part[s * stride], in split order, with up to 16
// loads in flight (splits past S re-read split S - 1 and are dropped).
__device__ __forceinline__ double sum_strided(const double *part, int64_t stride, int S) {
    constexpr int SB = 16;
    double acc = 0.0;
    for (int s0 = 0; s0 < S; s0 += SB) {
        double t[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) t[u] = part[(int64_t)(s0 + u < S ? s0 + u : S - 1) * stride];
#pragma unroll
        for (int u = 0; u < SB; ++u) acc += (s0 + u < S) ? t[u] : 0.0;
    }
    return acc;
}

// The whole X-half in one kernel (grid Tn tiles x Sx column splits): every
// block streams its split of the tile's 64 rows.  With one split the tile's
// rows of B_X are complete after the stream; with several, each block stores
// its partial and the tile's last block to arrive (per-tile counter) sums the
// partials in split order.  That block's first wave then solves the rows (one
// per lane) and writes the tile's statistics and G_X record (the X-side
// records number Rx = Tn).
template <int K, int P>
__device__ __forceinline__ void xfused_body(const AnlsParams &p, int tile, int split, double *lds) {
    const bool stop = sweep_stopped(p);
    __shared__ double G[K * K];
    __shared__ double scr[STHR];
    __shared__ unsigned flag;
    const double gacc = records_partial(p.gy_part, p.Ry, K * K, (int)threadIdx.x, STHR);
    const int64_t j0 = (int64_t)split * p.xcols;
    const int64_t j1 = min(j0 + (int64_t)p.xcols, p.m);
    if (!xstream_sums<K, P>(p, tile, j0, j1, lds, stop)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)tile * XTILE + lane;
    const bool live = i < p.n;
    const int64_t ic = live ? i : p.n - 1;
    double b[K];
#pragma unroll
    for (int a = 0; a < K; ++a) b[a] = 0.0;
    if (p.Sx > 1) {
        if (w == 0 && live) {
#pragma unroll
            for (int a = 0; a < K; ++a) {
                double v = lds[(0 * K + a) * XTILE + lane];
#pragma unroll
                for (int ww = 1; ww < SWAVES; ++ww) v += lds[(ww * K + a) * XTILE + lane];
                p.bx_part[((int64_t)split * K + a) * p.ldX + i] = v;
            }
        }
        if (!last_arrival(p.tile_cnt + tile, (unsigned)p.Sx, &flag)) return;
        if (w == 0) sum_split_partials<K>(p.bx_part, p.ldX, ic, p.Sx, b);
    } else if (w == 0) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double v = lds[(0 * K + a) * XTILE + lane];
#pragma unroll
            for (int ww = 1; ww < SWAVES; ++ww) v += lds[(ww * K + a) * XTILE + lane];
            b[a] = 0.0 + v;
        }
    }
    records_finish(gacc, K * K, 0, STHR, G, scr);
    if (w != 0) return;
    double x[K], st[NST], xn[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        x[a] = p.X[(int64_t)a * p.ldX + ic];
        xn[a] = 0.0;
    }
    const uint32_t old_mask = p.xmask[ic];
#pragma unroll
    for (int q = 0; q < NST; ++q) st[q] = 0.0;
    if (live) x_row<K>(p, G, i, x, b, old_mask, st, xn);
    wave_stats_and_gram<K>(st, xn, p.xstat + (int64_t)tile * NST,
                           p.mode == 0 ? p.gx_part + (int64_t)tile * K * K : nullptr);
}

template <int K>
__device__ __forceinline__ void xnnls_body(const AnlsParams &p, int bid) {
    constexpr int NT = nnls_threads(K);
    __shared__ double G[K * K];
    __shared__ double lds[NT];
    const bool stop = sweep_stopped(p);
    const int64_t i = (int64_t)bid * NT + threadIdx.x;
    const bool live = i < p.n;
    // the row's loads and the G_Y records go out before anything waits on
    // memory; lanes past the last row load row n - 1 and solve nothing
    const int64_t ic = live ? i : p.n - 1;
    double b[K], x[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        b[a] = 0.0;
        x[a] = p.X[(int64_t)a * p.ldX + ic];
    }
    const uint32_t old_mask = p.xmask[ic];
    sum_split_partials<K>(p.bx_part, p.ldX, ic, p.Sx, b);
    const double gacc = records_partial(p.gy_part, p.Ry, K * K, (int)threadIdx.x, NT);
    if (stop) return;
    records_finish(gacc, K * K, 0, NT, G, lds);
    double st[NST];
#pragma unroll
    for (int q = 0; q < NST; ++q) st[q] = 0.0;
    double xn[K];
#pragma unroll
    for (int a = 0; a < K; ++a) xn[a] = 0.0;
    if (live) x_row<K>(p, G, i, x, b, old_mask, st, xn);
    // the wave's record; with four-wave blocks, waves wholly past the last
    // row have none (the branch is uniform within a wave)
    const int64_t wv = i / WTHR;
    if (wv < p.Wx)
        wave_stats_and_gram<K>(st, xn, p.xstat + wv * NST, p.mode == 0 ? p.gx_part + wv * K * K : nullptr);
}

// ---------------------------------------------------------------- Y-half
// Streams the rows [r0, r1) of the tile's J = 64 / K columns of M against X
// and leaves each wave's transpose-reduced sums in red[w * YVALS + lane]
// (value jj * K + a is B_Y[a][jb + jj]); ends with a barrier.  With `stop`
// set the block returns false before any load.  For k >= 5 each lane takes
// two adjacent rows at a time with 16-byte loads (8-byte for the 4-byte copies
// of M), which halves the load instructions: a row costs k loads of X beside
// the J = 64/k loads of M, as many at k = 8.  r0 is even (row splits are
// multiples of 64 rows), so every pair load is aligned.
template <int K, int P>
__device__ __forceinline__ bool ystream_sums(const AnlsParams &p, int ct, int64_t r0, int64_t r1, double *red,
                                             bool stop) {
    using T = typename MElem<P>::T;
    constexpr int J = YVALS / K;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t jb = (int64_t)ct * J;
    const int nj = (int)min((int64_t)J, p.m - jb);

    T v[YVALS];
#pragma unroll
    for (int q = 0; q < YVALS; ++q) v[q] = T(0);
    if (stop) return false;
    if constexpr (K <= 4) {
        // J >= 16 loads of M per row: one row per lane (row pairs measured
        // slower here, and at k <= 2 they would not fit the registers)
        for (int64_t i = r0 + threadIdx.x; i < r1; i += STHR) {
            const int64_t base = jb * p.ldM + i;
            T x[K], mv[J];
#pragma unroll
            for (int a = 0; a < K; ++a) x[a] = (T)p.X[(int64_t)a * p.ldX + i];
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
                const T e = MElem<P>::load(p, base + (int64_t)min(jj, nj - 1) * p.ldM);
                mv[jj] = jj < nj ? e : T(0);
            }
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
#pragma unroll
                for (int a = 0; a < K; ++a) v[jj * K + a] = fma(mv[jj], x[a], v[jj * K + a]);
            }
        }
    } else {
        for (int64_t i = r0 + 2 * (int64_t)threadIdx.x; i < r1; i += 2 * STHR) {
            // rows i and i + 1; the second is dropped past r1 (its loads stay
            // inside the padded leading dimensions, which hold n + 1 rows when n
            // is odd), and so are columns past the tile's last
            const bool two = i + 1 < r1;
            T x0[K], x1[K], m0[J], m1[J];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const double2 xv = *reinterpret_cast<const double2 *>(p.X + (int64_t)a * p.ldX + i);
                x0[a] = (T)xv.x;
                x1[a] = two ? (T)xv.y : T(0);
            }
            const int64_t base = jb * p.ldM + i;
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
                T e0, e1;
                MElem<P>::load2(p, base + (int64_t)min(jj, nj - 1) * p.ldM, e0, e1);
                m0[jj] = jj < nj ? e0 : T(0);
                m1[jj] = (jj < nj && two) ? e1 : T(0);
            }
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    v[jj * K + a] = fma(m0[jj], x0[a], v[jj * K + a]);
                    v[jj * K + a] = fma(m1[jj], x1[a], v[jj * K + a]);
                }
            }
        }
    }
    red[w * YVALS + lane] = (double)wave_transpose_reduce(v, lane);
    __syncthreads();
    return true;
}

// Y stream, one row split: partial sums of B_Y for the split.
template <int K, int P>
__device__ __forceinline__ void ystream_body(const AnlsParams &p, int ct, int split) {
    const bool stop = sweep_stopped(p);
    constexpr int J = YVALS / K;
    __shared__ double red[SWAVES * YVALS];
    const int64_t r0 = (int64_t)split * p.yrows;
    const int64_t r1 = min(r0 + (int64_t)p.yrows, p.n);
    if (!ystream_sums<K, P>(p, ct, r0, r1, red, stop)) return;
    const int64_t jb = (int64_t)ct * J;
    const int nj = (int)min((int64_t)J, p.m - jb);
    if ((int)threadIdx.x < nj * K) {
        double s = red[threadIdx.x];
#pragma unroll
        for (int ww = 1; ww < SWAVES; ++ww) s += red[ww * YVALS + threadIdx.x];
        const int jj = threadIdx.x / K, a = threadIdx.x - jj * K;
        p.by_part[((int64_t)split * K + a) * p.ldY + jb + jj] = s;
    }
}

// The whole Y-half in one kernel (grid Tm tiles x Sy row splits): every block
// streams its split of the tile's J columns.  With one split the tile's
// columns of B_Y are complete after the stream; with several, each block
// stores its partial and the tile's last block to arrive (per-tile counter)
// sums the partials in split order.  That block's first wave then solves the
// columns (one per lane), writes the tile's statistics and G_Y record (the
// Y-side records number Ry = Tm), and the tile that finishes last closes the
// sweep.
template <int K, int P>
__device__ __forceinline__ void yfused_body(const AnlsParams &p, int ct, int split) {
    const bool stop = sweep_stopped(p);
    constexpr int J = YVALS / K;
    __shared__ double red[SWAVES * YVALS];
    __shared__ double G[K * K];
    __shared__ double scr[STHR];
    __shared__ double bsum[YVALS];
    __shared__ unsigned flag;
    const double gacc = records_partial(p.gx_part, p.Rx, K * K, (int)threadIdx.x, STHR);
    const int64_t r0 = (int64_t)split * p.yrows;
    const int64_t r1 = min(r0 + (int64_t)p.yrows, p.n);
    if (!ystream_sums<K, P>(p, ct, r0, r1, red, stop)) return;
    const int64_t jb = (int64_t)ct * J;
    const int nj = (int)min((int64_t)J, p.m - jb);
    const int t = (int)threadIdx.x;
    if (p.Sy > 1) {
        if (t < nj * K) {
            double s = red[t];
#pragma unroll
            for (int ww = 1; ww < SWAVES; ++ww) s += red[ww * YVALS + t];
            const int jj = t / K, a = t - jj * K;
            p.by_part[((int64_t)split * K + a) * p.ldY + jb + jj] = s;
        }
        if (!last_arrival(p.tile_cnt + p.Tn + ct, (unsigned)p.Sy, &flag)) return;
        if (t < nj * K) {
            const int jj = t / K, a = t - jj * K;
            bsum[t] = sum_strided(p.by_part + (int64_t)a * p.ldY + jb + jj, (int64_t)K * p.ldY, p.Sy);
        }
    } else if (t < nj * K) {
        double s = red[t];
#pragma unroll
        for (int ww = 1; ww < SWAVES; ++ww) s += red[ww * YVALS + t];
        bsum[t] = 0.0 + s;
    }
    records_finish(gacc, K * K, 0, STHR, G, scr);   // its barriers also publish bsum
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w == 0) {
        const bool live = lane < nj;
        const int64_t j = jb + lane;
        double b[K], y[K], st[NST], yn[K];
        uint32_t old_mask = 0u;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            b[a] = live ? bsum[lane * K + a] : 0.0;
            y[a] = live ? p.Y[(int64_t)a * p.ldY + j] : 0.0;
            yn[a] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < NST; ++q) st[q] = 0.0;
        if (live) {
            old_mask = p.ymask[j];
            y_col<K>(p, G, j, y, b, old_mask, st, yn);
        }
        wave_stats_and_gram<K>(st, yn, p.ystat + (int64_t)ct * NST, p.gy_part + (int64_t)ct * K * K);
    }
    if (!last_arrival(p.cnt_fin, (unsigned)p.Tm, &flag)) return;
    sweep_summary(p, scr);
}

template <int K>
__device__ __forceinline__ void ynnls_body(const AnlsParams &p, int bid) {
    constexpr int NT = nnls_threads(K);
    __shared__ double G[K * K];
    __shared__ double lds[NT];
    __shared__ unsigned flag;
    const bool stop = sweep_stopped(p);
    const int64_t j = (int64_t)bid * NT + threadIdx.x;
    const bool live = j < p.m;
    // the column's loads and the G_X records go out before anything waits on
    // memory; lanes past the last column load column m - 1 and solve nothing
    const int64_t jc = live ? j : p.m - 1;
    double b[K], y[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        b[a] = 0.0;
        y[a] = p.Y[(int64_t)a * p.ldY + jc];
    }
    const uint32_t old_mask = p.ymask[jc];
    sum_split_partials<K>(p.by_part, p.ldY, jc, p.Sy, b);
    const double gacc = records_partial(p.gx_part, p.Rx, K * K, (int)threadIdx.x, NT);
    if (stop) return;
    records_finish(gacc, K * K, 0, NT, G, lds);
    double st[NST];
#pragma unroll
    for (int q = 0; q < NST; ++q) st[q] = 0.0;
    double yn[K];
#pragma unroll
    for (int a = 0; a < K; ++a) yn[a] = 0.0;
    if (live) y_col<K>(p, G, j, y, b, old_mask, st, yn);
    const int64_t wv = j / WTHR;   // the wave's record (none past the last column)
    if (wv < p.Wy) wave_stats_and_gram<K>(st, yn, p.ystat + wv * NST, p.gy_part + wv * K * K);
    if (!last_arrival(p.cnt_fin, (unsigned)p.Ny, &flag)) return;
    sweep_summary(p, lds);
}

// ---------------------------------------------------------------- kernels
// One problem: the grid is the problem's own launch shape.
template <int K, int P>
__global__ __launch_bounds__(STHR) void k_xstream(AnlsParams p) {
    __shared__ double lds[xstream_lds<K>()];
    xstream_body<K, P>(p, blockIdx.x, blockIdx.y, lds);
}
template <int K, int P>
__global__ __launch_bounds__(STHR) void k_xfused(AnlsParams p) {
    __shared__ double lds[xstream_lds<K>()];
    xfused_body<K, P>(p, blockIdx.x, blockIdx.y, lds);
}
template <int K, int P>
__global__ __launch_bounds__(STHR) void k_yfused(AnlsParams p) { yfused_body<K, P>(p, blockIdx.x, blockIdx.y); }
template <int K>
__global__ __launch_bounds__(nnls_threads(K)) void k_xnnls(AnlsParams p) { xnnls_body<K>(p, blockIdx.x); }
template <int K, int P>
__global__ __launch_bounds__(STHR) void k_ystream(AnlsParams p) { ystream_body<K, P>(p, blockIdx.x, blockIdx.y); }
template <int K>
__global__ __launch_bounds__(nnls_threads(K)) void k_ynnls(AnlsParams p) { ynnls_body<K>(p, blockIdx.x); }

// A batch of problems with the same K and precision: one flattened grid, block
// b belongs to the problem q with off[q] <= b < off[q + 1] and runs that
// problem's block b - off[q] of its own launch shape.  off is non-decreasing
// with off[0] = 0, so q is the last index with off[q] <= b (problems without
// blocks in this kernel are skipped).  Each wave finds it on its own: 64 lanes
// probe 64 evenly spaced entries of the remaining range and a ballot keeps
// the last probe that is <= b, so np <= 64 takes one load per lane and
// np <= 4096 two, where a binary search would chain log2(np) loads.
__device__ __forceinline__ int batch_problem(const int *off, int np, int b) {
    const int lane = threadIdx.x & 63;
    int lo = 0, span = np;   // the answer is in [lo, lo + span); off[lo] <= b
    while (span > 1) {
        const int step = (span + 63) / 64;
        const int idx = lo + lane * step;
        const bool ok = idx < lo + span && off[idx < np ? idx : np - 1] <= b;
        const unsigned long long mask = __ballot(ok);
        const int last = 63 - __clzll((long long)mask);   // lane 0 always probes off[lo] <= b
        lo += last * step;
        span = min(step, span - last * step);
    }
    return lo;
}

template <int K, int P>
__global__ __launch_bounds__(STHR) void kb_xstream(const AnlsParams *tab, const int *off, int np) {
    const int q = batch_problem(off, np, blockIdx.x);
    const AnlsParams p = tab[q];
    const int local = blockIdx.x - off[q];
    __shared__ double lds[xstream_lds<K>()];
    xstream_body<K, P>(p, local % p.Tn, local / p.Tn, lds);
}
template <int K, int P>
__global__ __launch_bounds__(STHR) void kb_xfused(const AnlsParams *tab, const int *off, int np) {
    const int q = batch_problem(off, np, blockIdx.x);
    const AnlsParams p = tab[q];
    __shared__ double lds[xstream_lds<K>()];
    const int local = blockIdx.x - off[q];
    xfused_body<K, P>(p, local % p.Tn, local / p.Tn, lds);
}
template <int K>
__global__ __launch_bounds__(nnls_threads(K)) void kb_xnnls(const AnlsParams *tab, const int *off, int np) {
    const int q = batch_problem(off, np, blockIdx.x);
    const AnlsParams p = tab[q];
    xnnls_body<K>(p, blockIdx.x - off[q]);
}
template <int K, int P>
__global__ __launch_bounds__(STHR) void kb_ystream(const AnlsParams *tab, const int *off, int np) {
    const int q = batch_problem(off, np, blockIdx.x);
    const AnlsParams p = tab[q];
    const int local = blockIdx.x - off[q];
    ystream_body<K, P>(p, local % p.Tm, local / p.Tm);
}
template <int K, int P>
__global__ __launch_bounds__(STHR) void kb_yfused(const AnlsParams *tab, const int *off, int np) {
    const int q = batch_problem(off, np, blockIdx.x);
    const AnlsParams p = tab[q];
    const int local = blockIdx.x - off[q];
    yfused_body<K, P>(p, local % p.Tm, local / p.Tm);
}
template <int K>
__global__ __launch_bounds__(nnls_threads(K)) void kb_ynnls(const AnlsParams *tab, const int *off, int np) {
    const int q = batch_problem(off, np, blockIdx.x);
    const AnlsParams p = tab[q];
    ynnls_body<K>(p, blockIdx.x - off[q]);
}

// E(.;0) at the current iterate after a measure-mode k_xnnls: X part from the
// block records, Y part from the last Y-half.
template <int K>
__global__ __launch_bounds__(NTHR) void k_measure_finish(AnlsParams p) {
    __shared__ double sx[NST];
    __shared__ double scr[NTHR];
    reduce_records(p.xstat, p.Rx, NST, sx, scr);
    if (threadIdx.x == 0) {
        DevStatus *st = p.st;
        const double yg = st->ey_g2 >= 0.0 ? st->ey_g2 : 0.0;
        const double yc = st->ey_c2 >= 0.0 ? st->ey_c2 : 0.0;
        const double eg = sqrt(sx[ST_EG2] + yg);
        const double ec = sqrt(sx[ST_EC2] + yc);
        st->E_cur = eg > ec ? eg : ec;
    }
}

// G_Y records from the current Y, Ry of them (block b covers ceil(m / Ry)
// <= 256 columns), as the Y-half writes them.
template <int K>
__global__ __launch_bounds__(NTHR) void k_gram_y_init(AnlsParams p) {
    __shared__ double ys[NTHR * K];
    const int64_t per = (p.m + p.Ry - 1) / p.Ry;
    const int64_t j = (int64_t)blockIdx.x * per + threadIdx.x;
    const bool on = threadIdx.x < per && j < p.m;
#pragma unroll
    for (int a = 0; a < K; ++a) ys[threadIdx.x * K + a] = on ? p.Y[(int64_t)a * p.ldY + j] : 0.0;
    __syncthreads();
    for (int q = threadIdx.x; q < K * K; q += NTHR) {
        const int a = q / K, c = q - a * K;
        double v = 0.0;
        for (int l = 0; l < NTHR; ++l) v = fma(ys[l * K + a], ys[l * K + c], v);
        p.gy_part[(int64_t)blockIdx.x * K * K + q] = v;
    }
}

// G_X records from the current X, Rx of them (block b covers ceil(n / Rx)
// <= 256 rows), as the X-half writes them.
template <int K>
__global__ __launch_bounds__(NTHR) void k_gram_x_init(AnlsParams p) {
    __shared__ double xs[NTHR * K];
    const int64_t per = (p.n + p.Rx - 1) / p.Rx;
    const int64_t i = (int64_t)blockIdx.x * per + threadIdx.x;
    const bool on = threadIdx.x < per && i < p.n;
#pragma unroll
    for (int a = 0; a < K; ++a) xs[threadIdx.x * K + a] = on ? p.X[(int64_t)a * p.ldX + i] : 0.0;
    __syncthreads();
    for (int q = threadIdx.x; q < K * K; q += NTHR) {
        const int a = q / K, c = q - a * K;
        double v = 0.0;
        for (int l = 0; l < NTHR; ++l) v = fma(xs[l * K + a], xs[l * K + c], v);
        p.gx_part[(int64_t)blockIdx.x * K * K + q] = v;
    }
}

// Direct objective 1/2 ||XY - M||^2: per-block partials, fixed order.
template <int K>
__global__ __launch_bounds__(NTHR) void k_objective(AnlsParams p, double *part) {
    __shared__ double red[NTHR];
    double acc = 0.0;
    const int64_t total = p.n * p.m;
    for (int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x; e < total; e += (int64_t)gridDim.x * NTHR) {
        const int64_t j = e / p.n, i = e - j * p.n;
        double r = -p.M[j * p.ldM + i];
#pragma unroll
        for (int a = 0; a < K; ++a) r = fma(p.X[(int64_t)a * p.ldX + i], p.Y[(int64_t)a * p.ldY + j], r);
        acc = fma(r, r, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = NTHR / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
    __shared__ unsigned flag;
    if (!last_arrival(p.cnt_fin + 1, gridDim.x, &flag)) return;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b) s += part[b];
        p.st->f_direct = 0.5 * s;
    }
}

// part[0..nblk): ||M||^2 partials; part[nblk..2 nblk): count of non-finite entries.
__global__ __launch_bounds__(NTHR) void k_check_finite(const double *M, int64_t n, int64_t m, int64_t ldM,
                                                       double *part) {
    __shared__ double red[NTHR], bad[NTHR];
    double acc = 0.0, nb = 0.0;
    const int64_t total = n * m;
    for (int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x; e < total; e += (int64_t)gridDim.x * NTHR) {
        const int64_t j = e / n, i = e - j * n;
        const double v = M[j * ldM + i];
        if (isfinite(v)) acc = fma(v, v, acc);
        else nb += 1.0;
    }
    red[threadIdx.x] = acc;
    bad[threadIdx.x] = nb;
    __syncthreads();
    for (int h = NTHR / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[threadIdx.x] += red[threadIdx.x + h];
            bad[threadIdx.x] += bad[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = red[0];
        part[gridDim.x + blockIdx.x] = bad[0];
    }
}

// Row-major X (n x K) and Y (K x m) into the component-major device layout;
// masks from the signs.  Either source may be NULL (left untouched).
// Negative or non-finite entries are counted in *bad.
template <int K>
__global__ void k_factor_in(const double *sx, const double *sy, AnlsParams p, unsigned *bad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned nb = 0;
    if (sx && e < p.n) {
        uint32_t P = 0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const double v = sx[e * K + a];
            p.X[(int64_t)a * p.ldX + e] = v;
            if (v > 0.0) P |= 1u << a;
            if (!(v >= 0.0) || !isfinite(v)) ++nb;
        }
        p.xmask[e] = P;
    }
    if (sy && e < p.m) {
        uint32_t P = 0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const double v = sy[(int64_t)a * p.m + e];
            p.Y[(int64_t)a * p.ldY + e] = v;
            if (v > 0.0) P |= 1u << a;
            if (!(v >= 0.0) || !isfinite(v)) ++nb;
        }
        p.ymask[e] = P;
    }
    if (nb) atomicAdd(bad, nb);
}

template <int K>
__global__ void k_factor_out(AnlsParams p, double *dx, double *dy) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (dx && e < p.n) {
#pragma unroll
        for (int a = 0; a < K; ++a) dx[e * K + a] = p.X[(int64_t)a * p.ldX + e];
    }
    if (dy && e < p.m) {
#pragma unroll
        for (int a = 0; a < K; ++a) dy[(int64_t)a * p.m + e] = p.Y[(int64_t)a * p.ldY + e];
    }
}

// The 4-byte copy of columns [j0, j1) of M: FP32 (round to nearest), or the
// BF16 high part (round to nearest of the FP32 value) with the BF16 of the
// remainder in the low half.
__global__ __launch_bounds__(NTHR) void k_make_lowprec(AnlsParams p, int64_t j0, int64_t j1) {
    const int64_t total = p.n * (j1 - j0);
    for (int64_t e = (int64_t)blockIdx.x * NTHR + threadIdx.x; e < total; e += (int64_t)gridDim.x * NTHR) {
        const int64_t j = j0 + e / p.n, i = e % p.n;
        const int64_t off = j * p.ldM + i;
        const float f = (float)p.M[off];
        uint32_t out;
        if (p.prec == NMF_GRAM_FP32) {
            out = __float_as_uint(f);
        } else {
            const uint32_t u = __float_as_uint(f);
            const uint32_t hi = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;   // round to nearest even
            const float rem = f - __uint_as_float(hi);
            const uint32_t ur = __float_as_uint(rem);
            const uint32_t lo = ((ur + 0x7FFFu + ((ur >> 16) & 1u)) >> 16) & 0xFFFFu;
            out = hi | lo;
        }
        const_cast<uint32_t *>(p.Mlo)[off] = out;
    }
}

// Columns [j0, j1) of Y start from column j_from and its passive set (the
// neighbouring-column warm start for appended time instants).
template <int K>
__global__ void k_copy_columns_warm(AnlsParams p, int64_t j_from, int64_t j0, int64_t j1) {
    const int64_t j = j0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= j1) return;
#pragma unroll
    for (int a = 0; a < K; ++a) p.Y[(int64_t)a * p.ldY + j] = p.Y[(int64_t)a * p.ldY + j_from];
    p.ymask[j] = p.ymask[j_from];
}

__global__ void k_rearm(DevStatus *st, int budget) {
    if (threadIdx.x == 0) {
        st->converged = 0;
        st->max_sweeps = st->sweeps + budget;
    }
}

__global__ void k_batch_poll(const AnlsParams *table, int count, long long *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const DevStatus *st = table[q].st;
    out[2 * q] = st->converged;
    out[2 * q + 1] = st->sweeps;
}

// ---------------------------------------------------------------- tables of the grouped solves
// Marks the warm-start passive set of every problem of the half.
__global__ __launch_bounds__(256) void k_gmark(AnlsParams p, int yhalf) {
    if (sweep_stopped(p)) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (yhalf ? p.m : p.n)) return;
    p.gpresent[yhalf ? p.ymask[i] : p.xmask[i]] = 1;
}

// Numbers the marked sets in increasing order (one block), records each
// set's slot, and clears the marks for the next half.
__global__ __launch_bounds__(1024) void k_gnumber(AnlsParams p, int K) {
    __shared__ int cnt[1024];
    if (sweep_stopped(p)) return;
    const int NM = 1 << K, per = (NM + 1023) / 1024;
    const int m0 = min((int)threadIdx.x * per, NM), m1 = min(m0 + per, NM);
    int c = 0;
    for (int q = m0; q < m1; ++q) c += p.gpresent[q] ? 1 : 0;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = (int)threadIdx.x >= off ? cnt[threadIdx.x - off] : 0;
        __syncthreads();
        cnt[threadIdx.x] += v;
        __syncthreads();
    }
    int slot = cnt[threadIdx.x] - c;
    for (int q = m0; q < m1; ++q) {
        if (p.gpresent[q]) {
            if (slot < p.gcap) {
                p.gslot[q] = slot;
                p.gmask[slot] = (uint32_t)q;
            } else {
                p.gslot[q] = -1;
            }
            ++slot;
            p.gpresent[q] = 0;
        }
    }
    if (threadIdx.x == 1023) *p.gcount = min(cnt[1023], p.gcap);
}

// (G_PP)^-1 for each numbered set, one wave per set.  G is summed from the
// half's records exactly as the solve kernel sums it.  The matrix that is
// factored is G on P x P and the identity elsewhere; lane r < K holds row r of
// the factor (right-looking, one pivot broadcast per step) and, in the same
// steps, column r of W = L^-1; the inverse is W^T W, kept on P x P.
template <int K>
__global__ __launch_bounds__(nnls_threads(K)) void k_ginverse(AnlsParams p, int yhalf) {
    constexpr int NT = nnls_threads(K);
    __shared__ double G[K * K];
    __shared__ double lds[NT];
    if (sweep_stopped(p)) return;
    const int count = *p.gcount;
    const int slot0 = blockIdx.x * (NT / 64);
    if (slot0 >= count) return;
    const double gacc = yhalf ? records_partial(p.gx_part, p.Rx, K * K, (int)threadIdx.x, NT)
                              : records_partial(p.gy_part, p.Ry, K * K, (int)threadIdx.x, NT);
    records_finish(gacc, K * K, 0, NT, G, lds);
    const int slot = slot0 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (slot >= count) return;
    const uint32_t P = p.gmask[slot];
    const int r = lane < K ? lane : K - 1;
    const bool pr = (P >> r) & 1u;
    double a[K], w[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        a[c] = (pr && ((P >> c) & 1u)) ? G[r * K + c] : (r == c ? 1.0 : 0.0);
        w[c] = (c == r) ? 1.0 : 0.0;
    }
    double dmin = 1.0, dsum = 0.0;   // the sum catches NaN and infinite pivots, which fmin drops
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const double d = lane_bcast(a[c], c);
        dmin = fmin(dmin, d);
        dsum += d;
        const double s = rsqrt_newton(d > 0.0 ? d : 1.0);
        const double l = a[c] * s;
        a[c] = l;
        w[c] *= s;
#pragma unroll
        for (int jj = c + 1; jj < K; ++jj) {
            const double ljc = lane_bcast(l, jj);
            a[jj] = fma(-l, ljc, a[jj]);
            w[jj] = fma(-ljc, w[c], w[jj]);
            asm volatile("" : "+v"(w[jj]));
        }
    }
    const bool bad = !(dmin > 0.0) || !isfinite(dsum);
    double *T = p.gtab + (int64_t)slot * (K * K);
#pragma unroll
    for (int bcol = 0; bcol < K; ++bcol) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) v = fma(w[q], lane_bcast(w[q], bcol), v);
        if (lane < K)
            T[r * K + bcol] = bad ? __builtin_nan("") : ((pr && ((P >> bcol) & 1u)) ? v : 0.0);
    }
}

// ---------------------------------------------------------------- launchers
#define NMF_K_SWITCH(K, CALL)                                                        \
    switch (K) {                                                                     \
        case 1: { constexpr int KK = 1; CALL; } break;                               \
        case 2: { constexpr int KK = 2; CALL; } break;                               \
        case 3: { constexpr int KK = 3; CALL; } break;                               \
        case 4: { constexpr int KK = 4; CALL; } break;                               \
        case 5: { constexpr int KK = 5; CALL; } break;                               \
        case 6: { constexpr int KK = 6; CALL; } break;                               \
        case 7: { constexpr int KK = 7; CALL; } break;                               \
        case 8: { constexpr int KK = 8; CALL; } break;                               \
        case 9: { constexpr int KK = 9; CALL; } break;                               \
        case 10: { constexpr int KK = 10; CALL; } break;                             \
        case 11: { constexpr int KK = 11; CALL; } break;                             \
        case 12: { constexpr int KK = 12; CALL; } break;                             \
        case 13: { constexpr int KK = 13; CALL; } break;                             \
        case 14: { constexpr int KK = 14; CALL; } break;                             \
        case 15: { constexpr int KK = 15; CALL; } break;                             \
        case 16: { constexpr int KK = 16; CALL; } break;                             \
        default: return hipErrorInvalidValue;                                        \
    }

int yhalf_cols(int K) { return K >= 1 && K <= KMAX ? YVALS / K : 0; }

hipError_t launch_xstream(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (p.fx) {   // stream and solve in one kernel
        const dim3 g(p.Tn, p.Sx);
        if (p.prec == NMF_GRAM_FP32) {
            NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_xfused<KK, NMF_GRAM_FP32>), g, dim3(STHR), 0, s, e0, e1, 0, p));
        } else if (p.prec == NMF_GRAM_BF16X2) {
            NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_xfused<KK, NMF_GRAM_BF16X2>), g, dim3(STHR), 0, s, e0, e1, 0, p));
        } else {
            NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_xfused<KK, NMF_GRAM_FP64>), g, dim3(STHR), 0, s, e0, e1, 0, p));
        }
        return hipGetLastError();
    }
    const dim3 g(p.Tn, p.Sx);
    if (p.prec == NMF_GRAM_FP32) {
        NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_xstream<KK, NMF_GRAM_FP32>), g, dim3(STHR), 0, s, e0, e1, 0, p));
    } else if (p.prec == NMF_GRAM_BF16X2) {
        NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_xstream<KK, NMF_GRAM_BF16X2>), g, dim3(STHR), 0, s, e0, e1, 0, p));
    } else {
        NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_xstream<KK, NMF_GRAM_FP64>), g, dim3(STHR), 0, s, e0, e1, 0, p));
    }
    return hipGetLastError();
}

hipError_t launch_group_table(int K, const AnlsParams &p, int yhalf, hipStream_t s) {
    if (K < 1 || K > KMAX) return hipErrorInvalidValue;
    const int64_t cnt = yhalf ? p.m : p.n;
    hipLaunchKernelGGL(k_gmark, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, yhalf);
    hipLaunchKernelGGL(k_gnumber, dim3(1), dim3(1024), 0, s, p, K);
    const int per = nnls_threads(K) / 64;
    const unsigned blocks = (unsigned)((p.gcap + per - 1) / per);
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_ginverse<KK>, dim3(blocks), dim3(nnls_threads(KK)), 0, s, p, yhalf));
    return hipGetLastError();
}

hipError_t launch_xnnls(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (p.fx) return hipSuccess;   // solved inside k_xfused
    if (p.grouped && p.mode == 0) {
        const hipError_t e = launch_group_table(K, p, 0, s);
        if (e != hipSuccess) return e;
    }
    NMF_K_SWITCH(K, hipExtLaunchKernelGGL(k_xnnls<KK>, dim3(p.Nx), dim3(nnls_threads(KK)), 0, s, e0, e1, 0, p));
    return hipGetLastError();
}

hipError_t launch_ystream(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (p.fy) {   // stream and solve in one kernel
        const dim3 g(p.Tm, p.Sy);
        if (p.prec == NMF_GRAM_FP32) {
            NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_yfused<KK, NMF_GRAM_FP32>), g, dim3(STHR), 0, s, e0, e1, 0, p));
        } else if (p.prec == NMF_GRAM_BF16X2) {
            NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_yfused<KK, NMF_GRAM_BF16X2>), g, dim3(STHR), 0, s, e0, e1, 0, p));
        } else {
            NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_yfused<KK, NMF_GRAM_FP64>), g, dim3(STHR), 0, s, e0, e1, 0, p));
        }
        return hipGetLastError();
    }
    const dim3 g(p.Tm, p.Sy);
    if (p.prec == NMF_GRAM_FP32) {
        NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_ystream<KK, NMF_GRAM_FP32>), g, dim3(STHR), 0, s, e0, e1, 0, p));
    } else if (p.prec == NMF_GRAM_BF16X2) {
        NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_ystream<KK, NMF_GRAM_BF16X2>), g, dim3(STHR), 0, s, e0, e1, 0, p));
    } else {
        NMF_K_SWITCH(K, hipExtLaunchKernelGGL((k_ystream<KK, NMF_GRAM_FP64>), g, dim3(STHR), 0, s, e0, e1, 0, p));
    }
    return hipGetLastError();
}

hipError_t launch_ynnls(int K, const AnlsParams &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (p.fy) return hipSuccess;   // solved inside k_yfused
    if (p.grouped) {
        const hipError_t e = launch_group_table(K, p, 1, s);
        if (e != hipSuccess) return e;
    }
    NMF_K_SWITCH(K, hipExtLaunchKernelGGL(k_ynnls<KK>, dim3(p.Ny), dim3(nnls_threads(KK)), 0, s, e0, e1, 0, p));
    return hipGetLastError();
}

hipError_t launch_xhalf(int K, const AnlsParams &p, hipStream_t s) {
    hipError_t e = launch_xstream(K, p, s);
    return e != hipSuccess ? e : launch_xnnls(K, p, s);
}

hipError_t launch_yhalf(int K, const AnlsParams &p, hipStream_t s) {
    hipError_t e = launch_ystream(K, p, s);
    return e != hipSuccess ? e : launch_ynnls(K, p, s);
}

hipError_t launch_batch_sweep(int K, int prec, const BatchGroup &g, hipStream_t s) {
    if (g.count == 1) {
        hipError_t e = launch_xhalf(K, g.single, s);
        return e != hipSuccess ? e : launch_yhalf(K, g.single, s);
    }
    const AnlsParams *t = g.table;
    const int *o = g.off;
    const int np = g.count;
    const int *ox = o, *onx = o + (np + 1), *oy = o + 2 * (np + 1), *ony = o + 3 * (np + 1);
    const int *ofx = o + 4 * (np + 1), *ofy = o + 5 * (np + 1);
#define NMF_BATCH_STREAM(KERNEL, NB, OFF)                                                                      \
    if ((NB) > 0) {                                                                                           \
        if (prec == NMF_GRAM_FP32) {                                                                          \
            NMF_K_SWITCH(K, hipLaunchKernelGGL((KERNEL<KK, NMF_GRAM_FP32>), dim3(NB), dim3(STHR), 0, s, t, OFF, np)); \
        } else if (prec == NMF_GRAM_BF16X2) {                                                                 \
            NMF_K_SWITCH(K, hipLaunchKernelGGL((KERNEL<KK, NMF_GRAM_BF16X2>), dim3(NB), dim3(STHR), 0, s, t, OFF, np)); \
        } else {                                                                                              \
            NMF_K_SWITCH(K, hipLaunchKernelGGL((KERNEL<KK, NMF_GRAM_FP64>), dim3(NB), dim3(STHR), 0, s, t, OFF, np)); \
        }                                                                                                     \
    }
    // X-half: split streams, fused halves, then the row NNLS of the split ones
    NMF_BATCH_STREAM(kb_xstream, g.blocks[0], ox)
    NMF_BATCH_STREAM(kb_xfused, g.blocks[4], ofx)
    if (g.blocks[1] > 0)
        NMF_K_SWITCH(K, hipLaunchKernelGGL(kb_xnnls<KK>, dim3(g.blocks[1]), dim3(nnls_threads(KK)), 0, s, t, onx, np));
    // Y-half
    NMF_BATCH_STREAM(kb_ystream, g.blocks[2], oy)
    NMF_BATCH_STREAM(kb_yfused, g.blocks[5], ofy)
    if (g.blocks[3] > 0)
        NMF_K_SWITCH(K, hipLaunchKernelGGL(kb_ynnls<KK>, dim3(g.blocks[3]), dim3(nnls_threads(KK)), 0, s, t, ony, np));
#undef NMF_BATCH_STREAM
    return hipGetLastError();
}

hipError_t launch_measure_finish(int K, const AnlsParams &p, hipStream_t s) {
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_measure_finish<KK>, dim3(1), dim3(NTHR), 0, s, p));
    return hipGetLastError();
}

hipError_t launch_gram_y_init(int K, const AnlsParams &p, hipStream_t s) {
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_gram_y_init<KK>, dim3(p.Ry), dim3(NTHR), 0, s, p));
    return hipGetLastError();
}

hipError_t launch_gram_x_init(int K, const AnlsParams &p, hipStream_t s) {
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_gram_x_init<KK>, dim3(p.Rx), dim3(NTHR), 0, s, p));
    return hipGetLastError();
}

hipError_t launch_objective(int K, const AnlsParams &p, double *part, int nblk, hipStream_t s) {
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_objective<KK>, dim3(nblk), dim3(NTHR), 0, s, p, part));
    return hipGetLastError();
}

hipError_t launch_check_finite(const double *M, int64_t n, int64_t m, int64_t ldM, double *part, int nblk,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(nblk), dim3(NTHR), 0, s, M, n, m, ldM, part);
    return hipGetLastError();
}

static dim3 grid_rows(const AnlsParams &p) {
    const int64_t e = p.n > p.m ? p.n : p.m;
    return dim3((unsigned)((e + NTHR - 1) / NTHR));
}

hipError_t launch_factor_in(int K, const double *sx, const double *sy, const AnlsParams &p, unsigned *bad,
                            hipStream_t s) {
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_factor_in<KK>, grid_rows(p), dim3(NTHR), 0, s, sx, sy, p, bad));
    return hipGetLastError();
}

hipError_t launch_factor_out(int K, const AnlsParams &p, double *dx, double *dy, hipStream_t s) {
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_factor_out<KK>, grid_rows(p), dim3(NTHR), 0, s, p, dx, dy));
    return hipGetLastError();
}

hipError_t launch_make_lowprec(const AnlsParams &p, int64_t j0, int64_t j1, hipStream_t s) {
    if (p.prec == NMF_GRAM_FP64 || j1 <= j0) return hipSuccess;
    hipLaunchKernelGGL(k_make_lowprec, dim3(1024), dim3(NTHR), 0, s, p, j0, j1);
    return hipGetLastError();
}

hipError_t launch_rearm(DevStatus *st, int budget, hipStream_t s) {
    hipLaunchKernelGGL(k_rearm, dim3(1), dim3(64), 0, s, st, budget);
    return hipGetLastError();
}

hipError_t launch_batch_poll(const AnlsParams *table, int count, long long *out, hipStream_t s) {
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_batch_poll, dim3((unsigned)((count + NTHR - 1) / NTHR)), dim3(NTHR), 0, s, table, count, out);
    return hipGetLastError();
}

hipError_t launch_copy_columns_warm(int K, const AnlsParams &p, int64_t j_from, int64_t j0, int64_t j1,
                                    hipStream_t s) {
    if (j1 <= j0) return hipSuccess;
    const unsigned nb = (unsigned)((j1 - j0 + NTHR - 1) / NTHR);
    NMF_K_SWITCH(K, hipLaunchKernelGGL(k_copy_columns_warm<KK>, dim3(nb), dim3(NTHR), 0, s, p, j_from, j0, j1));
    return hipGetLastError();
}

}  // namespace nmfk
