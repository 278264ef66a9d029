// Dense linear algebra of the interior-point stage (Sec. III-B, eq. (20)):
// formation of the Gauss-Newton Schur complement, its Cholesky factorisation
// and the two triangular solves, on FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Ordering of S.  The unknowns dy are ordered component-major, row a*m + j for
// Y_aj.  Then S = Q2bar - sum_i (x_i x_i^T) (x) C_i with C_i[j][l] =
// Y_j^T Q1bar_i^-1 Y_l = Z_i[:, j] . Z_i[:, l] (Z_i = L_i^-1 Y): the k x k grid
// of m x m blocks, block (a, b) = sum_i X_ia X_ib C_i, is symmetric block by
// block, so one product C_i[J, L] of a 16 x 16 tile pair (J >= L) serves
// every (a, b) with a >= b and its mirrored tile.
//
// S is stored column-major with leading dimension ldS >= NT*64 and padded to
// NT*64 rows and columns with the identity, so every kernel works on whole
// 64 x 64 tiles.  Only the lower triangle is read.  After the factorisation
// the tiles below the diagonal hold L; the diagonal factor tiles are kept, as
// their inverses, in Dinv.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dense.h"

namespace nmfk {

typedef double v4d __attribute__((ext_vector_type(4)));

// D = A B + C on one 16 x 16 x 4 FP64 matrix-core step.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16]
// (v = 0..3; checked on the device).
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 1/sqrt(v) for v > 0: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double v) {
    double y = __builtin_amdgcn_rsq(v);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-v * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

__device__ __forceinline__ double lane_read(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

constexpr unsigned kSpinLimit = 1u << 24;   // ~1 s of polling, then give up and flag it

// Publishes flags[idx] = epoch after every store of the block (release,
// device scope).
__device__ __forceinline__ void post_flag(unsigned *flags, int idx, unsigned epoch) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(flags + idx, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------- Schur complement
// Tile pair index -> (jt, lt), jt >= lt, row-major over the lower triangle.
__device__ __forceinline__ void tri_pair(int64_t tp, int64_t &jt, int64_t &lt) {
    jt = (int64_t)((sqrt(8.0 * (double)tp + 1.0) - 1.0) * 0.5);
    while ((jt + 1) * (jt + 2) / 2 <= tp) ++jt;
    while (jt * (jt + 1) / 2 > tp) --jt;
    lt = tp - jt * (jt + 1) / 2;
}

// Packed index t of (a, b), a >= b: t = a (a + 1) / 2 + b.
__device__ __forceinline__ void tri_ab(int t, int &a, int &b) {
    a = 0;
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    b = t - a * (a + 1) / 2;
}

// Writes one 16 x 16 tile of block (a, b) of S (lane values in the matrix-
// core output layout) and, for a > b off the diagonal tile, its mirror; on
// the diagonal tile adds delta_jl Q2bar_j[a][b] = G_X[a][b] + delta_ab (rho +
// s_aj / y_aj).
template <int K>
__device__ __forceinline__ void schur_store(const SchurArgs &g, int64_t jt, int64_t lt, int a, int b, const double (&val)[4]) {
    const int lane = threadIdx.x & 63, gq = lane >> 4, r = lane & 15;
    const int64_t m = g.m;
    const int64_t l = lt * 16 + r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t j = jt * 16 + gq + 4 * v;
        if (j < m && l < m) {
            double x = val[v];
            if (jt == lt && j == l) {
                x = g.GX[a * K + b] - x;
                if (a == b) x += g.rho + g.s[(int64_t)a * g.ldY + j] / g.Y[(int64_t)a * g.ldY + j];
            } else {
                x = -x;
            }
            g.S[(b * m + l) * g.ldS + a * m + j] = x;
            if (a > b && jt != lt) g.S[(b * m + j) * g.ldS + a * m + l] = x;
        }
    }
}

// Work split of the Gauss-Newton formation for rank K: the K(K+1)/2 products
// (a, b) are summed in `nch` chunks (one wave per tile pair and chunk), Z
// operands of `ru` rows are prefetched, and X_ia X_ib of `ch` rows are staged
// per block.  Chosen as the fewest chunks whose accumulators, prefetched
// operands and staging registers fit 256 registers per lane (two waves per
// SIMD hide each other's load and matrix-core latency; at K = 10 that is 1.56x
// faster than one wave per SIMD with half the chunks), with `ch` rows of
// products at most 4 registers per thread.
struct GnPlan { int nch, ru, ch; };
constexpr GnPlan kGnPlan[17] = {
    {1, 4, 64}, {1, 4, 64}, {1, 4, 64}, {1, 4, 64}, {1, 4, 64}, {1, 4, 64}, {1, 2, 48}, {2, 4, 36}, {2, 2, 28},
    {3, 2, 20}, {4, 2, 16}, {4, 2, 12}, {5, 2, 12}, {6, 2, 8}, {7, 2, 8}, {8, 2, 8}, {8, 2, 4}};

// One wave per unit (tile pair, (a,b) chunk); the four waves of a block
// share a row split, whose rows i they sum of X_ia X_ib C_i[J, L], C_i[J, L]
// from KS matrix-core steps over the (zero-padded) components of Z_i.  The
// X_ia X_ib of CH rows at a time are staged in LDS (one copy per block,
// broadcast reads; the next chunk's are loaded into registers while the
// current chunk is summed, two LDS buffers, one barrier per chunk); the Z
// operands of the next RU rows are loaded while the current RU rows are summed,
// across chunk boundaries, and the matrix-core product of the next row is
// issued before the vector updates of the current one.
template <int K>
__global__ __launch_bounds__(256) void k_schur_gn(SchurArgs g) {
    constexpr int NL = K * (K + 1) / 2;
    constexpr int NCH = kGnPlan[K].nch;
    constexpr int CS = (NL + NCH - 1) / NCH;
    constexpr int KS = zpad(K) / 4;
    constexpr int RU = kGnPlan[K].ru;
    constexpr int CH = kGnPlan[K].ch;
    constexpr int XR = (CH * NL + 255) / 256;
    static_assert(CH % RU == 0, "row groups must not straddle chunks");
    __shared__ double xs[2][CH * NL];
    const int lane = threadIdx.x & 63, gq = lane >> 4, r = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int p = (int)(blockIdx.x % g.P);
    const int64_t wu = (int64_t)(blockIdx.x / g.P) * 4 + wave;
    const int64_t nunits = (int64_t)g.npairs * NCH;
    const bool active = wu < nunits;   // wave-uniform
    const int ch = active ? (int)(wu % NCH) : 0;
    const int64_t tp = active ? wu / NCH : 0;
    int64_t jt, lt;
    tri_pair(tp, jt, lt);
    const int64_t i0 = (int64_t)p * g.rows_per_split;
    const int64_t i1 = min(g.n, i0 + g.rows_per_split);
    const int t0 = ch * CS;
    int64_t offA[KS], offB[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        offA[s] = (int64_t)(gq + 4 * s) * g.ldY + jt * 16 + r;
        offB[s] = (int64_t)(gq + 4 * s) * g.ldY + lt * 16 + r;
    }
    const int64_t zstride = (int64_t)zpad(K) * g.ldY;
    double acc[CS][4];
#pragma unroll
    for (int t = 0; t < CS; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] = 0.0;
    if (i0 < i1) {   // block-uniform
        {
            const int nr = (int)min((int64_t)CH, i1 - i0);
            for (int idx = threadIdx.x; idx < nr * NL; idx += 256) xs[0][idx] = g.XX[i0 * NL + idx];
        }
        // operands of the current and the next RU rows (rows clamped into
        // the split: loads stay in range)
        double av[RU][KS], bv[RU][KS], an[RU][KS], bn[RU][KS];
        if (active) {
#pragma unroll
            for (int uu = 0; uu < RU; ++uu) {
                const double *zi = g.Z + min(i0 + uu, i1 - 1) * zstride;
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    av[uu][s] = zi[offA[s]];
                    bv[uu][s] = zi[offB[s]];
                }
            }
        }
        __syncthreads();
        int buf = 0;
        for (int64_t c0 = i0; c0 < i1; c0 += CH) {
            const int nr = (int)min((int64_t)CH, i1 - c0);
            const int64_t c1 = c0 + CH;
            const int nr1 = (int)max((int64_t)0, min((int64_t)CH, i1 - c1));
            double xn[XR];
#pragma unroll
            for (int q = 0; q < XR; ++q) {
                const int idx = (int)threadIdx.x + 256 * q;
                xn[q] = idx < nr1 * NL ? g.XX[c1 * NL + idx] : 0.0;
            }
            if (active) {
                const double *xb = xs[buf];
                for (int rb = 0; rb < nr; rb += RU) {
#pragma unroll
                    for (int uu = 0; uu < RU; ++uu) {
                        const double *zi = g.Z + min(c0 + rb + RU + uu, i1 - 1) * zstride;
#pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            an[uu][s] = zi[offA[s]];
                            bn[uu][s] = zi[offB[s]];
                        }
                    }
                    v4d cn = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s = 0; s < KS; ++s) cn = mfma16(av[0][s], bv[0][s], cn);
#pragma unroll
                    for (int uu = 0; uu < RU; ++uu) {
                        const v4d c = cn;
                        if (uu + 1 < RU) {
                            cn = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                            for (int s = 0; s < KS; ++s) cn = mfma16(av[uu + 1][s], bv[uu + 1][s], cn);
                        }
                        if (rb + uu < nr) {   // wave-uniform
                            const double *xr = xb + (rb + uu) * NL + t0;
#pragma unroll
                            for (int t = 0; t < CS; ++t) {
                                if (t0 + t < NL) {
                                    const double w = xr[t];
#pragma unroll
                                    for (int v = 0; v < 4; ++v) acc[t][v] = fma(c[v], w, acc[t][v]);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int uu = 0; uu < RU; ++uu)
#pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            av[uu][s] = an[uu][s];
                            bv[uu][s] = bn[uu][s];
                        }
                }
            }
            // the other buffer was last read in the previous chunk, before
            // the barrier that ended it
            buf ^= 1;
#pragma unroll
            for (int q = 0; q < XR; ++q) {
                const int idx = (int)threadIdx.x + 256 * q;
                if (idx < nr1 * NL) xs[buf][idx] = xn[q];
            }
            __syncthreads();
        }
    }
    if (!active) return;
    if (g.P == 1) {
#pragma unroll
        for (int t = 0; t < CS; ++t) {
            if (t0 + t < NL) {
                int a, b;
                tri_ab(t0 + t, a, b);
                schur_store<K>(g, jt, lt, a, b, acc[t]);
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < CS; ++t) {
            if (t0 + t < NL) {
                double *dst = g.part + (((int64_t)p * g.npairs + tp) * NL + t0 + t) * 256 + lane * 4;
#pragma unroll
                for (int v = 0; v < 4; ++v) dst[v] = acc[t][v];
            }
        }
    }
}

// Sums the row-split partials in split order and stores them into S; one
// wave per (tile pair, (a, b)).
template <int K>
__global__ __launch_bounds__(256) void k_schur_reduce(SchurArgs g) {
    constexpr int NL = K * (K + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= (int64_t)g.npairs * NL) return;
    const int t = (int)(u % NL);
    const int64_t tp = u / NL;
    double val[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = 0; p < g.P; ++p) {
        const double *src = g.part + (((int64_t)p * g.npairs + tp) * NL + t) * 256 + lane * 4;
#pragma unroll
        for (int v = 0; v < 4; ++v) val[v] += src[v];
    }
    int64_t jt, lt;
    tri_pair(tp, jt, lt);
    int a, b;
    tri_ab(t, a, b);
    schur_store<K>(g, jt, lt, a, b, val);
}

// Element type, matrix-core step and output layout of the exact-Hessian rank
// update: FP64, or FP32 for the mixed-precision form (V rounded to FP32; S
// itself, the factorisation and the solves stay FP64, and the direction is
// refined against the FP64 operator).
template <bool F32> struct MfmaT;
template <> struct MfmaT<false> {
    typedef double E;
    typedef v4d A;
    static __device__ __forceinline__ A mma(E a, E b, A c) { return mfma16(a, b, c); }
    // row of the output value v held by lane group gq
    static __device__ __forceinline__ int drow(int gq, int v) { return gq + 4 * v; }
};
template <> struct MfmaT<true> {
    typedef float E;
    typedef float A __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ A mma(E a, E b, A c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int drow(int gq, int v) { return 4 * gq + v; }   // checked on the device
};

// Rows [k0, k1) of the exact-Hessian factor (eq. (27)) written out once:
// V[k - k0][(a, j)] = X_ia Z_i[p][j] + (L_i^-1)[p][a] R_ij for k = i*K + p,
// columns in component-major order (a*m + j), zero from N = m K to ldV;
// rounded to FP32 for the mixed-precision form.
// Block x < cbm covers columns j = 256 x + t of every component a (Z_i[p][j]
// and R_ij loaded once for the K entries); the blocks after them zero the
// padding columns [N, ldV).  Each block writes VGEN_ROWS consecutive rows
// (few, larger blocks: the dispatch rate of tiny blocks, not HBM, bounded a
// one-row form).
constexpr int VGEN_ROWS = 8;
template <int K, typename E>
__global__ __launch_bounds__(256) void k_vgen(SchurExArgs g, int64_t k0, int64_t k1, E *V, int64_t ldV) {
    const int64_t N = g.m * K;
    const int cbm = (int)((g.m + 255) / 256);
    const int bx = (int)blockIdx.x;
    const int64_t kb = k0 + (int64_t)blockIdx.y * VGEN_ROWS;
    const int64_t ke = min(k1, kb + VGEN_ROWS);
    if (bx < cbm) {
        const int64_t j = (int64_t)bx * 256 + threadIdx.x;
        if (j >= g.m) return;
        for (int64_t k = kb; k < ke; ++k) {
            const int64_t i = k / K;
            const int p = (int)(k - i * K);
            const double z = g.Z[(i * zpad(K) + p) * g.ldY + j];
            const double rv = g.R[i * g.ldY + j];
            const double *li = g.Linv + (i * K + p) * K;
            E *vr = V + (k - k0) * ldV + j;
#pragma unroll
            for (int a = 0; a < K; ++a) vr[(int64_t)a * g.m] = (E)fma(g.X[(int64_t)a * g.ldX + i], z, li[a] * rv);
        }
    } else {
        const int64_t c = N + (int64_t)(bx - cbm) * 256 + threadIdx.x;
        if (c >= ldV) return;
        for (int64_t k = kb; k < ke; ++k) V[(k - k0) * ldV + c] = (E)0.0;
    }
}

// Entry (x, y, v) of the lane's output blocks, summed over the rows: written
// into S (first: S = Q2bar - sum, else S -= sum).
template <int K, bool F32>
__device__ __forceinline__ void syrk_put(const SchurExArgs &g, int64_t It, int64_t Jt, int R0, int C0, int gq, int r,
                                         int x, int y, int v, double sum, int first) {
    typedef MfmaT<F32> M;
    const int64_t N = g.m * K;
    const int64_t row = It * 128 + R0 + 16 * x + r, cl = Jt * 128 + C0 + 16 * y + M::drow(gq, v);
    if (row < N && cl < N) {
        double *dst = g.S + cl * g.ldS + row;
        if (first) {
            const int a = (int)(row / g.m), b = (int)(cl / g.m);
            const int64_t j = row - a * g.m, l = cl - b * g.m;
            double val = -sum;
            if (j == l) {
                val += g.GX[a * K + b];
                if (a == b) val += g.rho + g.s[(int64_t)a * g.ldY + j] / g.Y[(int64_t)a * g.ldY + j];
            }
            *dst = val;
        } else {
            *dst -= sum;
        }
    }
}

// SPLIT: the rows of the slab are split over blockIdx.y (nsplit ranges of whole
// 16-row chunks) and each block writes its partial tile to kpart (entry q =
// (x*4 + y)*4 + v of thread t at ((s * tiles + tile) * 32 + q) * 512 + t);
// k_syrk_reduce then sums the splits in order and writes S.
template <int K, bool F32, bool SPLIT>
__global__ __launch_bounds__(512) void k_syrk_v(SchurExArgs g, const typename MfmaT<F32>::E *V, int64_t ldV,
                                                int64_t rows, int first, int nsplit, double *kpart) {
    typedef MfmaT<F32> M;
    typedef typename M::E E;
    constexpr int TW = 128;                           // tile width
    constexpr int KC = 16;                            // rows of V per chunk
    constexpr int PER = 16 / (int)sizeof(E);          // elements per 16-byte load
    constexpr int TSH = KC * TW / PER;                // loads per tile and chunk
    constexpr int RSH = TW / PER;                     // loads per row of a tile
    constexpr int NLD = 2 * TSH / 512;                // loads per thread and chunk
    __shared__ __align__(16) E VA[2][KC * TW];
    __shared__ __align__(16) E VB[2][KC * TW];
    int64_t It, Jt;
    tri_pair(blockIdx.x, It, Jt);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63, gq = lane >> 4, r = lane & 15;
    const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 64;
    const bool work = !(It == Jt && R0 + 32 <= C0);   // wave-uniform
    int64_t kbeg = 0, kend = rows;
    if (SPLIT) {
        const int64_t per = ((rows + nsplit - 1) / nsplit + KC - 1) / KC * KC;
        kbeg = min(rows, (int64_t)blockIdx.y * per);
        kend = min(rows, kbeg + per);
    }
    uint4 ld[NLD];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int h = 0; h < NLD; ++h) {
            const int idx = h * 512 + threadIdx.x, tile = idx / TSH, rem = idx % TSH, kk = rem / RSH, cq = rem % RSH;
            const int64_t kr = k0 + kk, col = (tile ? Jt : It) * TW + PER * cq;
            ld[h] = (kr < kend && col < ldV) ? *reinterpret_cast<const uint4 *>(V + kr * ldV + col)
                                             : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int h = 0; h < NLD; ++h) {
            const int idx = h * 512 + threadIdx.x, tile = idx / TSH, rem = idx % TSH;
            *reinterpret_cast<uint4 *>((tile ? VB[buf] : VA[buf]) + rem * PER) = ld[h];
        }
    };
    typename M::A acc[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[x][y][v] = (E)0;
    load(kbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
        const bool more = k0 + KC < kend;
        if (more) load(k0 + KC);
        if (work) {
#pragma unroll
            for (int s = 0; s < KC / 4; ++s) {
                const int kk = 4 * s + gq;
                E av[2], bv[4];
#pragma unroll
                for (int x = 0; x < 2; ++x) av[x] = VA[buf][kk * TW + R0 + 16 * x + r];
#pragma unroll
                for (int y = 0; y < 4; ++y) bv[y] = VB[buf][kk * TW + C0 + 16 * y + r];
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = M::mma(bv[y], av[x], acc[x][y]);
            }
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    if (!work) return;
    if (SPLIT) {
        double *dst = kpart + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 32 * 512 + threadIdx.x;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) dst[((x * 4 + y) * 4 + v) * 512] = (double)acc[x][y][v];
        return;
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) syrk_put<K, F32>(g, It, Jt, R0, C0, gq, r, x, y, v, (double)acc[x][y][v], first);
}

// Sums the nsplit partial tiles of k_syrk_v in split order and writes S;
// the same thread layout (and output positions) as k_syrk_v.  Block
// (tile, qg) handles the entries q = 4 qg .. 4 qg + 3 of its threads, so the
// partials are read by many blocks at once.
template <int K, bool F32>
__global__ __launch_bounds__(512) void k_syrk_reduce(SchurExArgs g, const double *kpart, int nsplit, int first) {
    int64_t It, Jt;
    tri_pair(blockIdx.x, It, Jt);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63, gq = lane >> 4, r = lane & 15;
    const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 64;
    if (It == Jt && R0 + 32 <= C0) return;
    const double *src = kpart + (int64_t)blockIdx.x * 32 * 512 + threadIdx.x;
    const int64_t sstride = (int64_t)gridDim.x * 32 * 512;
    const int q0 = (int)blockIdx.y * 4;
    double sum[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) sum[u] = src[(q0 + u) * 512];
    for (int s = 1; s < nsplit; ++s) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = src[s * sstride + (q0 + u) * 512];
#pragma unroll
        for (int u = 0; u < 4; ++u) sum[u] += t[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = q0 + u, x = q >> 4, y = (q >> 2) & 3, v = q & 3;
        syrk_put<K, F32>(g, It, Jt, R0, C0, gq, r, x, y, v, sum[u], first);
    }
}

// Linv[i][p][a] = (L_i^-1)[p][a], one row i per thread.
template <int K>
__global__ __launch_bounds__(256) void k_linv(const double *Lq, int64_t ldX, int64_t n, double *Linv) {
    constexpr int NL = K * (K + 1) / 2;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double L[NL], id[K];
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] = Lq[(int64_t)q * ldX + i];
#pragma unroll
    for (int a = 0; a < K; ++a) id[a] = Lq[(int64_t)(NL + a) * ldX + i];
    // column c of L^-1 by forward substitution from e_c
#pragma unroll
    for (int c = 0; c < K; ++c) {
        double x[K];
#pragma unroll
        for (int rr = 0; rr < K; ++rr) {
            double v = (rr == c) ? 1.0 : 0.0;
#pragma unroll
            for (int q = 0; q < rr; ++q) v -= L[rr * (rr + 1) / 2 + q] * x[q];
            x[rr] = v * id[rr];
        }
#pragma unroll
        for (int pq = 0; pq < K; ++pq) Linv[(i * K + pq) * K + c] = x[pq];
    }
}

// R[i*ldY + j] = (X Y - M)_ij by 32 x 32 tiles transposed through LDS (M is
// column-major, R row-major).
template <int K>
__global__ __launch_bounds__(256) void k_residual_rows(const double *M, int64_t ldM, const double *X, int64_t ldX,
                                                       const double *Y, int64_t ldY, int64_t n, int64_t m,
                                                       double *R) {
    __shared__ double tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        double v = 0.0;
        if (i < n && j < m) {
            v = -M[j * ldM + i];
#pragma unroll
            for (int a = 0; a < K; ++a) v = fma(X[(int64_t)a * ldX + i], Y[(int64_t)a * ldY + j], v);
        }
        tile[jj][tx] = v;
    }
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t i = i0 + ii, j = j0 + tx;
        if (i < n && j < ldY) R[i * ldY + j] = tile[tx][ii];
    }
}

// XX[i][t] = X_ia X_ib for t = (a, b), a >= b.
template <int K>
__global__ __launch_bounds__(256) void k_xx(const double *X, int64_t ldX, int64_t n, double *XX) {
    constexpr int NL = K * (K + 1) / 2;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double x[K];
#pragma unroll
    for (int a = 0; a < K; ++a) x[a] = X[(int64_t)a * ldX + i];
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) XX[i * NL + a * (a + 1) / 2 + b] = x[a] * x[b];
}

// Identity in the padding rows and columns [N, Np) of S (lower triangle).
__global__ __launch_bounds__(256) void k_pad_identity(double *S, int64_t ldS, int64_t N, int64_t Np) {
    const int64_t col = blockIdx.x;   // 0 .. Np-1
    for (int64_t row = N + threadIdx.x; row < Np; row += 256) {
        if (row >= col) S[col * ldS + row] = (row == col) ? 1.0 : 0.0;
    }
}

// ------------------------------------------------------------- Schur operator
// res = rhs - S v with S applied without forming it, in FP64: S = Q2bar -
// sum_i V_i^T V_i, V_i[p][(a, j)] = X_ia Z_i[p][j] (+ (L_i^-1)[p][a] R_ij for the
// exact Hessian, eq. (27)).  Used to refine a direction solved with a factor
// of an S formed in FP32.
// Pass 1, one block per row i: q = V_i v (K values), then t_i = Z_i^T q (row
// i of T) and h_i = L_i^-T q (exact).
template <int K, bool EXACT>
__global__ __launch_bounds__(256) void k_op_rows(OpArgs g) {
    constexpr int KP = zpad(K);
    __shared__ double red[4][2 * K];
    __shared__ double qs[K];
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double xi[K];
#pragma unroll
    for (int a = 0; a < K; ++a) xi[a] = g.X[(int64_t)a * g.ldX + i];
    const double *Zi = g.Z + i * KP * g.ldY;
    const double *Ri = g.R + i * g.ldY;
    double qz[K], rv[K];
#pragma unroll
    for (int a = 0; a < K; ++a) qz[a] = rv[a] = 0.0;
    for (int64_t j = threadIdx.x; j < g.m; j += 256) {
        double va[K], wv = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            va[a] = g.v[(int64_t)a * g.m + j];
            wv = fma(xi[a], va[a], wv);
        }
#pragma unroll
        for (int q = 0; q < K; ++q) qz[q] = fma(Zi[(int64_t)q * g.ldY + j], wv, qz[q]);
        if (EXACT) {
            const double rij = Ri[j];
#pragma unroll
            for (int a = 0; a < K; ++a) rv[a] = fma(rij, va[a], rv[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            qz[a] += __shfl_xor(qz[a], off);
            if (EXACT) rv[a] += __shfl_xor(rv[a], off);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            red[wave][a] = qz[a];
            red[wave][K + a] = rv[a];
        }
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int q = threadIdx.x;
        double v = red[0][q] + red[1][q] + red[2][q] + red[3][q];
        if (EXACT) {
            const double *li = g.Linv + (i * K + q) * K;
#pragma unroll
            for (int a = 0; a < K; ++a) v = fma(li[a], red[0][K + a] + red[1][K + a] + red[2][K + a] + red[3][K + a], v);
        }
        qs[q] = v;
    }
    __syncthreads();
    double qv[K];
#pragma unroll
    for (int q = 0; q < K; ++q) qv[q] = qs[q];
    for (int64_t l = threadIdx.x; l < g.ldY; l += 256) {
        double t = 0.0;
        if (l < g.m) {
#pragma unroll
            for (int q = 0; q < K; ++q) t = fma(Zi[(int64_t)q * g.ldY + l], qv[q], t);
        }
        g.T[i * g.ldY + l] = t;
    }
    if (EXACT && threadIdx.x < K) {
        const int a = threadIdx.x;
        double h = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) h = fma(g.Linv[(i * K + q) * K + a], qv[q], h);
        g.H[i * K + a] = h;
    }
}

// Pass 2: part[s][a][l] = sum over the rows i of split s of X_ia t_i[l]
// (+ h_i[a] R_il), one thread per column l.
template <int K, bool EXACT>
__global__ __launch_bounds__(256) void k_op_cols(OpArgs g) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int sp = blockIdx.y;
    const int64_t per = (g.n + g.S - 1) / g.S;
    const int64_t i0 = (int64_t)sp * per, i1 = min(g.n, i0 + per);
    if (l >= g.m) return;
    double acc[K];
#pragma unroll
    for (int a = 0; a < K; ++a) acc[a] = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double t = g.T[i * g.ldY + l];
#pragma unroll
        for (int a = 0; a < K; ++a) acc[a] = fma(g.X[(int64_t)a * g.ldX + i], t, acc[a]);
        if (EXACT) {
            const double rr = g.R[i * g.ldY + l];
#pragma unroll
            for (int a = 0; a < K; ++a) acc[a] = fma(g.H[i * K + a], rr, acc[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < K; ++a) g.part[((int64_t)sp * K + a) * g.ldY + l] = acc[a];
}

// Pass 3: res = rhs - (Q2bar v - sum_i V_i^T V_i v), zero past N.
template <int K>
__global__ __launch_bounds__(256) void k_op_residual(OpArgs g) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.Np) return;
    const int64_t N = g.m * K;
    if (e >= N) {
        g.res[e] = 0.0;
        return;
    }
    const int a = (int)(e / g.m);
    const int64_t l = e - (int64_t)a * g.m;
    double out = 0.0;
    for (int sp = 0; sp < g.S; ++sp) out += g.part[((int64_t)sp * K + a) * g.ldY + l];
    double q2 = (g.rho + g.s[(int64_t)a * g.ldY + l] / g.Y[(int64_t)a * g.ldY + l]) * g.v[e];
#pragma unroll
    for (int b = 0; b < K; ++b) q2 = fma(g.GX[a * K + b], g.v[(int64_t)b * g.m + l], q2);
    g.res[e] = g.rhs[e] - (q2 - out);
}

__global__ void k_axpy(double *y, const double *x, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < count) y[e] += x[e];
}

// ------------------------------------------------------------- Cholesky of S
constexpr int LDT = 65;   // LDS row stride (doubles) of a 64 x 64 tile

// Block column j of the factor of the 64 x 64 tile T (row-major, stride LDT)
// as one tall panel (rows 16 j .. 63, columns 16 j .. 16 j + 15), by one wave:
// lane p holds row 16 j + p in a[]; step c takes pivot c from lane c, scales
// column c and applies it to the row's later columns (right-looking), so the
// rows below the diagonal block (the sub-panels L_ij, i > j) come out of the
// same broadcasts as the diagonal block L_jj.  Lanes above a step's row
// compute values of the upper triangle that nothing reads, so no step needs a
// lane mask.  The column goes to Lf (L_jj with zeros above its diagonal).  A
// pivot that is not positive, or not finite, sets *bad (the factor is then
// not used) and is replaced by 1.
__device__ __forceinline__ void potrf_panel16(const double *T, double *Lf, int j, int *bad) {
    const int lane = threadIdx.x & 63;
    const int rows = 64 - 16 * j;
    const int p = lane < rows ? lane : rows - 1;
    const double *Trow = T + (16 * j + p) * LDT + 16 * j;
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = Trow[q];
    // fmin drops a NaN operand, so the pivots are also summed: a NaN or an
    // infinity among them makes the sum non-finite
    double dmin = 1.0, dsum = 0.0;
    double d = lane_read(a[0], 0);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        dmin = fmin(dmin, d);
        dsum += d;
        const double s = rsqrt_nr(d > 0.0 ? d : 1.0);
        const double l = a[c] * s;   // row p of column c; on lane c, sqrt(d)
        a[c] = l;
        if (c + 1 < 16) {
            // the next pivot first: lane c+1 updates its own diagonal entry with
            // its own l (the value every other lane receives by broadcast), so
            // the chain of pivots carries one broadcast per step
            const int c1 = c + 1 < 16 ? c + 1 : 15;
            const double dn = fma(-l, l, a[c1]);
            d = lane_read(dn, c1);
        }
#pragma unroll
        for (int jj = c + 1; jj < 16; ++jj) a[jj] = fma(-l, lane_read(l, jj), a[jj]);
    }
    if (lane < rows) {
        double *Lrow = Lf + (16 * j + p) * LDT + 16 * j;
#pragma unroll
        for (int q = 0; q < 16; ++q) Lrow[q] = (p >= 16 || q <= p) ? a[q] : 0.0;
    }
    if ((!(dmin > 0.0) || !isfinite(dsum)) && lane == 0) *bad = 1;
}

// W = L_jj^-1 for the 16 x 16 diagonal block j of the factor in Lf (lower,
// zeros above), by one wave: lane q < 16 solves L w = e_q by forward
// substitution (the entries of L are read by every lane alike, one LDS
// broadcast each).  W goes to the diagonal block j of T, which the
// factorisation no longer reads.
__device__ __forceinline__ void inverse16(double *T, const double *Lf, int j) {
    const int q = threadIdx.x & 15;
    const double *L = Lf + (16 * j) * LDT + 16 * j;
    double w[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        double v = (p == q) ? 1.0 : 0.0;
#pragma unroll
        for (int r = 0; r < p; ++r) v = fma(-L[p * LDT + r], w[r], v);
        w[p] = v / L[p * LDT + p];
    }
    if ((threadIdx.x & 63) < 16) {
#pragma unroll
        for (int p = 0; p < 16; ++p) T[(16 * j + p) * LDT + 16 * j + q] = w[p];
    }
}

// T_il -= L_ij L_lj^T for j < l <= i (one wave, row block i), with the
// sub-panels from Lf.  The product is formed transposed (D[q][p] = X[p][q]).
__device__ __forceinline__ void panel_update(double *T, const double *Lf, int j, int i) {
    const int lane = threadIdx.x & 63, gq = lane >> 4, r = lane & 15;
    double li[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) li[s] = Lf[(16 * i + r) * LDT + 16 * j + 4 * s + gq];
    for (int l = j + 1; l <= i; ++l) {
        double *Tb = T + (16 * i + r) * LDT + 16 * l + gq;
        v4d acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = Tb[4 * v];
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mfma16(-Lf[(16 * l + r) * LDT + 16 * j + 4 * s + gq], li[s], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) Tb[4 * v] = acc[v];
    }
}

// Step kt (-1 .. NT-2) of the right-looking factorisation by 64-wide block
// columns, for column c = kt + 1; 512 threads per block.
//   Tiles right of column c (c < tj <= ti): A_ij -= L_i,kt L_j,kt^T, in 2 x 2
//   groups of tiles per block, each of the 8 waves a 32 x 64 part.
//   Tiles of column c (blocks 0 .. NT-c-1, tile (c + b, c)): waves 0-3 update
//   their own tile, rows 16 w each (kt >= 0); waves 4-7 update the diagonal
//   tile (c, c) and factor it in LDS, 16-wide block column by block column
//   (every such block does the same arithmetic, so every copy of the factor is
//   identical).  Then waves 0-3 solve their rows of L_ic = A_ic L_cc^-T block
//   column by block column: X_y = (A_y - sum_{r<y} X_r L_yr^T) W_yy^T, with
//   W_yy the inverse of the 16 x 16 diagonal block.  Block 0 (the diagonal
//   tile) runs the same solve on the identity, which gives L_cc^-1 for the
//   triangular solves (Dinv[c]); tile (c, c) of S is not written.
// No block waits for another.
__global__ __launch_bounds__(512, 4) void k_chol_step(CholArgs g, int kt) {
    // T: the diagonal tile being factored; Lf: the factor's sub-blocks.  While
    // the update runs, the same memory holds the tile-column-kt panels.
    __shared__ __align__(16) double sm[2 * 64 * LDT];
    double *const T = sm, *const Lf = sm + 64 * LDT;
    const int c = kt + 1;
    const int NT = g.NT;
    const int bid = blockIdx.x;
    const int npanel = NT - c;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, gq = lane >> 4, r = lane & 15;
    double *S = g.S;
    const int64_t ldS = g.ldS;
    const int64_t db = (int64_t)c * 64, kb = (int64_t)kt * 64;
    // acc[..][v] is tile entry (16 x + r, 16 y + gq + 4 v): products are formed
    // transposed (D = L_j L_i^T block by block), so that 16 lanes hold 16
    // consecutive rows of one column.
    if (bid >= npanel) {
        // trailing tiles c < tj <= ti < NT in 2 x 2 groups (128 x 128: each
        // panel entry is loaded for two tiles), groups column by column; wave w
        // updates rows 32 (w % 4) and columns 64 (w / 4) of the group, which lie
        // in one tile (skipped past the last tile or above the diagonal)
        const int G = (NT - c) / 2;   // groups per side: ceil((NT - c - 1) / 2)
        int rr = bid - npanel, GJ = 0;
        while (rr >= G - GJ) {
            rr -= G - GJ;
            ++GJ;
        }
        const int GI = GJ + rr;
        const int R0 = (wave & 3) * 32, C0 = (wave >> 2) * 64;
        const int ti = c + 1 + 2 * GI + (R0 >> 6), tj = c + 1 + 2 * GJ + (C0 >> 6);
        if (ti >= NT || tj >= NT || ti < tj) return;
        const int64_t rb = (int64_t)ti * 64 + (R0 & 63), cb = (int64_t)tj * 64;
        v4d acc[2][4];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[x][y][v] = S[(cb + 16 * y + gq + 4 * v) * ldS + rb + 16 * x + r];
        // two matrix-core k-steps per group, the next group loaded ahead
        double qa[2][2][4], qb[2][2][2];
#pragma unroll
        for (int h = 0; h < 9; ++h) {
            if (h < 8) {
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const double *col = S + (kb + 8 * h + 4 * s2 + gq) * ldS;
#pragma unroll
                    for (int x = 0; x < 2; ++x) qb[h & 1][s2][x] = -col[rb + 16 * x + r];
#pragma unroll
                    for (int y = 0; y < 4; ++y) qa[h & 1][s2][y] = col[cb + 16 * y + r];
                }
            }
            if (h > 0) {
                const int hb = (h - 1) & 1;
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int y = 0; y < 4; ++y) acc[x][y] = mfma16(qa[hb][s2][y], qb[hb][s2][x], acc[x][y]);
            }
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) S[(cb + 16 * y + gq + 4 * v) * ldS + rb + 16 * x + r] = acc[x][y][v];
        return;
    }
    const int ti = c + bid;
    const int64_t rb = (int64_t)ti * 64;
    const bool diag = ti == c;
    const bool own = wave < 4;                 // waves 0-3: own tile; 4-7: tile (c, c)
    const int x = wave & 3;
    const int64_t tb = own ? rb : db;          // first row of the tile this wave updates
    v4d acc[4];
    if (own && diag) {
        // block 0, waves 0-3: the identity, whose solve gives L_cc^-1
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[y][v] = (16 * x + r == 16 * y + gq + 4 * v) ? 1.0 : 0.0;
    } else {
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[y][v] = S[(db + 16 * y + gq + 4 * v) * ldS + tb + 16 * x + r];
    }
    if (kt >= 0) {
        // acc -= L_t,kt L_c,kt^T over the 64 columns of tile column kt.  The
        // panels L_c,kt (P[0 ..]) and L_i,kt (P[4096 ..]; the same panel again
        // in block 0) are staged in LDS column by column (P[k*64 + row]) with
        // 16-byte loads.
        double *const P = sm;
        double2 st[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int idx = h * 512 + threadIdx.x, pan = idx >> 11, rem = idx & 2047, k = rem >> 5, rp = rem & 31;
            st[h] = *reinterpret_cast<const double2 *>(S + (kb + k) * ldS + (pan ? rb : db) + 2 * rp);
        }
#pragma unroll
        for (int h = 0; h < 8; ++h)
            *reinterpret_cast<double2 *>(P + ((h * 512 + threadIdx.x) & 4095) * 2) = st[h];
        __syncthreads();
        if (!(own && diag)) {
            // operands of k-step s4 + 1 are read from LDS while step s4 runs
            const double *Pb = P + (own ? 4096 : 0) + 16 * x + r + gq * 64;
            const double *Pa = P + r + gq * 64;
            double ca[4], cbv = Pb[0], na[4], nb = 0.0;
#pragma unroll
            for (int y = 0; y < 4; ++y) ca[y] = Pa[16 * y];
#pragma unroll
            for (int s4 = 0; s4 < 16; ++s4) {
                if (s4 + 1 < 16) {
                    nb = Pb[(s4 + 1) * 256];
#pragma unroll
                    for (int y = 0; y < 4; ++y) na[y] = Pa[(s4 + 1) * 256 + 16 * y];
                }
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[y] = mfma16(ca[y], -cbv, acc[y]);
#pragma unroll
                for (int y = 0; y < 4; ++y) ca[y] = na[y];
                cbv = nb;
            }
        }
        __syncthreads();
    }
    if (!own) {
        // the updated diagonal tile into T (lower 16 x 16 blocks)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            if (y <= x)
#pragma unroll
                for (int v = 0; v < 4; ++v) T[(16 * x + r) * LDT + 16 * y + gq + 4 * v] = acc[y][v];
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
        if (wave == 4 + j) potrf_panel16(T, Lf, j, g.fail);
        __syncthreads();
        if (!own && x > j) panel_update(T, Lf, j, x);
        __syncthreads();
    }
    // inverses of the four diagonal blocks, one per panel wave, into T
    if (own) inverse16(T, Lf, x);
    __syncthreads();
    if (!own) return;
    v4d X[4];
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        v4d t = acc[y];
#pragma unroll
        for (int rr = 0; rr < y; ++rr)
#pragma unroll
            for (int s = 0; s < 4; ++s) t = mfma16(-Lf[(16 * y + r) * LDT + 16 * rr + 4 * s + gq], X[rr][s], t);
        v4d z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) z = mfma16(T[(16 * y + r) * LDT + 16 * y + 4 * s + gq], t[s], z);
        X[y] = z;
    }
    if (diag) {
        // X = L_cc^-T: Dinv[c] holds L_cc^-1 column-major, entry (row a, column b) at b * 64 + a
        double *D = g.Dinv + (int64_t)c * 4096;
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) D[(16 * x + r) * 64 + 16 * y + gq + 4 * v] = X[y][v];
        return;
    }
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) S[(db + 16 * y + gq + 4 * v) * ldS + rb + 16 * x + r] = X[y][v];
}

// ------------------------------------------------------------- triangular solves
// Thread 0 waits for flags[q] == epoch, then extends over the following
// flags of the range [q, end) (step dir = +1 or -1) that are already set, and
// returns (through LDS) the last ready index; one acquire fence covers them.
__device__ __forceinline__ int wait_run(const unsigned *flags, int q, int end, int dir, unsigned epoch, int *fail,
                                        int *s_last) {
    if (threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(flags + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                atomicExch(fail, 2);
                break;
            }
        }
        int h = q;
        while (h + dir != end &&
               __hip_atomic_load(flags + h + dir, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch)
            h += dir;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_last = h;
    }
    __syncthreads();
    return *s_last;
}

// Forward solve L y = b by 64-row tiles, one block per tile, in one launch:
// block t accumulates L_tq y_q for q < t as the y_q are published, then
// y_t = Dinv[t] (b_t - sum).  Blocks wait only on lower block indices.  The
// tile of L needed next is loaded before each wait.
__global__ __launch_bounds__(256) void k_trsv_fwd_lb(SolveArgs g) {
    __shared__ double red[4][64];
    __shared__ double vs[64];
    __shared__ int s_last;
    const int t = blockIdx.x;
    const int r = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t ldS = g.ldS;
    const double *Lrow = g.S + (int64_t)part * 16 * ldS + (int64_t)t * 64 + r;   // + q*64*ldS + u*ldS
    double acc = 0.0, Lp[16], Dv[16];
    // this tile's inverse diagonal block and right-hand side, loaded before
    // any wait
    const double *D = g.Dinv + (int64_t)t * 4096;
#pragma unroll
    for (int u = 0; u < 16; ++u) Dv[u] = D[(part * 16 + u) * 64 + r];
    const double bt = g.b[(int64_t)t * 64 + r];
    if (t > 0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) Lp[u] = Lrow[(int64_t)u * ldS];
    }
    int q = 0;
    while (q < t) {
        const int h = wait_run(g.flags, q, t, 1, g.epoch, g.fail, &s_last);
        for (; q <= h; ++q) {
            double Lc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) Lc[u] = Lp[u];
            if (q + 1 < t) {
#pragma unroll
                for (int u = 0; u < 16; ++u) Lp[u] = Lrow[((int64_t)(q + 1) * 64 + u) * ldS];
            }
            const double *yq = g.y + (int64_t)q * 64 + part * 16;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = fma(-Lc[u], yq[u], acc);
        }
        __syncthreads();
    }
    red[part][r] = acc;
    __syncthreads();
    if (part == 0) vs[r] = bt + ((red[0][r] + red[1][r]) + (red[2][r] + red[3][r]));
    __syncthreads();
    double w = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) w = fma(Dv[u], vs[part * 16 + u], w);
    __syncthreads();
    red[part][r] = w;
    __syncthreads();
    if (part == 0) g.y[(int64_t)t * 64 + r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
    post_flag(g.flags, t, g.epoch);
}

// Backward solve L^T x = y in place on y, tiles from the last up: block b
// serves tile t = NT-1-b and accumulates L_qt^T x_q for q > t as the x_q are
// published, then x_t = Dinv[t]^T (y_t - sum).
__global__ __launch_bounds__(256) void k_trsv_bwd_lb(SolveArgs g) {
    __shared__ double red[4][64];
    __shared__ double vs[64];
    __shared__ int s_last;
    const int NT = g.NT;
    const int t = NT - 1 - (int)blockIdx.x;
    const int r = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t ldS = g.ldS;
    const double *Lcol = g.S + ((int64_t)t * 64 + r) * ldS + part * 16;   // + q*64 + u
    double acc = 0.0, Lp[16], Dv[16];
    const double *D = g.Dinv + (int64_t)t * 4096 + (int64_t)r * 64 + part * 16;
#pragma unroll
    for (int u = 0; u < 16; ++u) Dv[u] = D[u];
    if (t < NT - 1) {
#pragma unroll
        for (int u = 0; u < 16; ++u) Lp[u] = Lcol[(int64_t)(NT - 1) * 64 + u];
    }
    int q = NT - 1;
    while (q > t) {
        const int h = wait_run(g.flags, q, t, -1, g.epoch, g.fail, &s_last);
        for (; q >= h; --q) {
            double Lc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) Lc[u] = Lp[u];
            if (q - 1 > t) {
#pragma unroll
                for (int u = 0; u < 16; ++u) Lp[u] = Lcol[(int64_t)(q - 1) * 64 + u];
            }
            const double *xq = g.y + (int64_t)q * 64 + part * 16;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = fma(-Lc[u], xq[u], acc);
        }
        __syncthreads();
    }
    red[part][r] = acc;
    __syncthreads();
    if (part == 0) vs[r] = g.y[(int64_t)t * 64 + r] + ((red[0][r] + red[1][r]) + (red[2][r] + red[3][r]));
    __syncthreads();
    double w = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) w = fma(Dv[u], vs[part * 16 + u], w);
    __syncthreads();
    red[part][r] = w;
    __syncthreads();
    if (part == 0) g.y[(int64_t)t * 64 + r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
    post_flag(g.flags, t, g.epoch);
}

// ------------------------------------------------------------- launchers
#define DENSE_K_SWITCH(K, CALL)                                  \
    switch (K) {                                                 \
        case 1: { constexpr int KK = 1; CALL; } break;           \
        case 2: { constexpr int KK = 2; CALL; } break;           \
        case 3: { constexpr int KK = 3; CALL; } break;           \
        case 4: { constexpr int KK = 4; CALL; } break;           \
        case 5: { constexpr int KK = 5; CALL; } break;           \
        case 6: { constexpr int KK = 6; CALL; } break;           \
        case 7: { constexpr int KK = 7; CALL; } break;           \
        case 8: { constexpr int KK = 8; CALL; } break;           \
        case 9: { constexpr int KK = 9; CALL; } break;           \
        case 10: { constexpr int KK = 10; CALL; } break;         \
        case 11: { constexpr int KK = 11; CALL; } break;         \
        case 12: { constexpr int KK = 12; CALL; } break;         \
        case 13: { constexpr int KK = 13; CALL; } break;         \
        case 14: { constexpr int KK = 14; CALL; } break;         \
        case 15: { constexpr int KK = 15; CALL; } break;         \
        case 16: { constexpr int KK = 16; CALL; } break;         \
        default: return hipErrorInvalidValue;                    \
    }

int schur_chunks(int K) {
    return (K >= 1 && K <= 16) ? kGnPlan[K].nch : 1;
}

hipError_t launch_xx(int K, const double *X, int64_t ldX, int64_t n, double *XX, hipStream_t st) {
    const dim3 grid((unsigned)((n + 255) / 256));
    DENSE_K_SWITCH(K, hipLaunchKernelGGL(k_xx<KK>, grid, dim3(256), 0, st, X, ldX, n, XX));
    return hipGetLastError();
}

hipError_t launch_schur_gn(int K, const SchurArgs &g, hipStream_t st) {
    const int64_t units = (int64_t)g.npairs * schur_chunks(K);
    const dim3 grid((unsigned)((units + 3) / 4 * g.P));
    DENSE_K_SWITCH(K, hipLaunchKernelGGL(k_schur_gn<KK>, grid, dim3(256), 0, st, g));
    if (g.P > 1) {
        const int64_t ru = (int64_t)g.npairs * (K * (K + 1) / 2);
        const dim3 rg((unsigned)((ru + 3) / 4));
        DENSE_K_SWITCH(K, hipLaunchKernelGGL(k_schur_reduce<KK>, rg, dim3(256), 0, st, g));
    }
    return hipGetLastError();
}

// Row splits per tile for the exact-Hessian rank update: the count s <= 12
// that minimises the per-CU share ceil(tiles s / 256) / s of whole tiles (plus
// a small charge per split for the partial tiles), within the capacity.
int syrk_splits(int64_t tiles, int64_t cap) {
    int best = 1;
    double bc = 1e300;
    for (int s = 1; s <= 12; ++s) {
        if (s > 1 && (double)s * (double)tiles * 32.0 * 512.0 > (double)cap) break;
        const double c = (double)((tiles * s + 255) / 256) / s + 0.004 * s;
        if (c < bc - 1e-12) {
            bc = c;
            best = s;
        }
    }
    return best;
}

hipError_t launch_schur_exact_rows(int K, const SchurExArgs &g, void *V, int64_t ldV, int64_t slab, bool f32,
                                   double *kpart, int64_t kpart_cap, hipStream_t st) {
    const int64_t nk = g.n * K;
    if (slab < 32 || slab > 65535 || ldV < (int64_t)g.NT * 64 || ldV % 64 != 0) return hipErrorInvalidValue;
    const int64_t T2 = (g.NT + 1) / 2;   // 128-wide tiles
    const int64_t tiles = T2 * (T2 + 1) / 2;
    const int ns = kpart ? syrk_splits(tiles, kpart_cap) : 1;
    const dim3 grid((unsigned)tiles, (unsigned)ns);
    for (int64_t k0 = 0; k0 < nk; k0 += slab) {
        const int64_t k1 = std::min(nk, k0 + slab);
        const int64_t cbm = (g.m + 255) / 256;
        const dim3 gv((unsigned)(cbm + (ldV - g.m * K + 255) / 256),
                      (unsigned)((k1 - k0 + VGEN_ROWS - 1) / VGEN_ROWS));
        const int first = k0 == 0 ? 1 : 0;
        if (f32) {
            float *Vf = (float *)V;
            DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_vgen<KK, float>), gv, dim3(256), 0, st, g, k0, k1, Vf, ldV));
            if (ns > 1) {
                DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_syrk_v<KK, true, true>), grid, dim3(512), 0, st, g,
                                                     (const float *)Vf, ldV, k1 - k0, first, ns, kpart));
                DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_syrk_reduce<KK, true>), dim3((unsigned)tiles, 8), dim3(512), 0, st,
                                                     g, (const double *)kpart, ns, first));
            } else {
                DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_syrk_v<KK, true, false>), grid, dim3(512), 0, st, g,
                                                     (const float *)Vf, ldV, k1 - k0, first, 1, (double *)nullptr));
            }
        } else {
            double *Vd = (double *)V;
            DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_vgen<KK, double>), gv, dim3(256), 0, st, g, k0, k1, Vd, ldV));
            if (ns > 1) {
                DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_syrk_v<KK, false, true>), grid, dim3(512), 0, st, g,
                                                     (const double *)Vd, ldV, k1 - k0, first, ns, kpart));
                DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_syrk_reduce<KK, false>), dim3((unsigned)tiles, 8), dim3(512), 0, st,
                                                     g, (const double *)kpart, ns, first));
            } else {
                DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_syrk_v<KK, false, false>), grid, dim3(512), 0, st, g,
                                                     (const double *)Vd, ldV, k1 - k0, first, 1, (double *)nullptr));
            }
        }
    }
    return hipGetLastError();
}

hipError_t launch_schur_apply(int K, bool exact, const OpArgs &g, hipStream_t st) {
    if (g.S < 1 || g.n < 1 || g.m < 1) return hipErrorInvalidValue;
    const dim3 gc((unsigned)((g.m + 255) / 256), (unsigned)g.S);
    if (exact) {
        DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_op_rows<KK, true>), dim3((unsigned)g.n), dim3(256), 0, st, g));
        DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_op_cols<KK, true>), gc, dim3(256), 0, st, g));
    } else {
        DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_op_rows<KK, false>), dim3((unsigned)g.n), dim3(256), 0, st, g));
        DENSE_K_SWITCH(K, hipLaunchKernelGGL((k_op_cols<KK, false>), gc, dim3(256), 0, st, g));
    }
    DENSE_K_SWITCH(K, hipLaunchKernelGGL(k_op_residual<KK>, dim3((unsigned)((g.Np + 255) / 256)), dim3(256), 0, st, g));
    return hipGetLastError();
}

hipError_t launch_axpy(double *y, const double *x, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, y, x, count);
    return hipGetLastError();
}

hipError_t launch_linv(int K, const double *Lq, int64_t ldX, int64_t n, double *Linv, hipStream_t st) {
    const dim3 grid((unsigned)((n + 255) / 256));
    DENSE_K_SWITCH(K, hipLaunchKernelGGL(k_linv<KK>, grid, dim3(256), 0, st, Lq, ldX, n, Linv));
    return hipGetLastError();
}

hipError_t launch_residual_rows(int K, const double *M, int64_t ldM, const double *X, int64_t ldX,
                                const double *Y, int64_t ldY, int64_t n, int64_t m, double *R, hipStream_t st) {
    const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((ldY + 31) / 32));
    DENSE_K_SWITCH(K, hipLaunchKernelGGL(k_residual_rows<KK>, grid, dim3(256), 0, st, M, ldM, X, ldX, Y, ldY, n, m,
                                         R));
    return hipGetLastError();
}

hipError_t launch_pad_identity(double *S, int64_t ldS, int64_t N, int64_t Np, hipStream_t st) {
    if (Np <= N) return hipSuccess;
    hipLaunchKernelGGL(k_pad_identity, dim3((unsigned)Np), dim3(256), 0, st, S, ldS, N, Np);
    return hipGetLastError();
}

hipError_t launch_cholesky(const CholArgs &g, hipStream_t st) {
    const int NT = g.NT;
    for (int kt = -1; kt <= NT - 2; ++kt) {
        const int c = kt + 1;
        const int G = (NT - c) / 2;   // 2 x 2 groups of trailing tiles per side
        const int64_t blocks = (int64_t)(NT - c) + (kt >= 0 ? (int64_t)G * (G + 1) / 2 : 0);
        hipLaunchKernelGGL(k_chol_step, dim3((unsigned)blocks), dim3(512), 0, st, g, kt);
    }
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs &fwd, const SolveArgs &bwd, hipStream_t st) {
    hipLaunchKernelGGL(k_trsv_fwd_lb, dim3((unsigned)fwd.NT), dim3(256), 0, st, fwd);
    hipLaunchKernelGGL(k_trsv_bwd_lb, dim3((unsigned)bwd.NT), dim3(256), 0, st, bwd);
    return hipGetLastError();
}

__global__ void k_fill_u32(unsigned *p, int64_t count, unsigned v) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < count) p[e] = v;
}

hipError_t launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

}  // namespace nmfk
