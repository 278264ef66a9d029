// Host runtime behind include/nmf.h: workspace layout, launch planning, the
// stage machine of Alg. 3 and the C entry points.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/nmf.h"
#include "ipm.h"
#include "nmf_internal.h"

using nmfk::AnlsParams;
using nmfk::DevStatus;

namespace {

constexpr int kRedBlocks = 512;   // blocks of the fixed-order reduction kernels
constexpr int kSxMax = 64;        // column splits of the X-half
constexpr int kSyMax = 64;        // row splits of the Y-half

thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Plan {
    int64_t ldM, ldX, ldY;
    int Tn, Sx, xcols, Sy, yrows, Tm, J, Bx, By, Nx, Ny, Wx, Wy;
    bool FX, FY;   // the half runs as one kernel
};

// Stage-1 launch shape.  X stream: 64-row tiles, column splits so that about
// 4096 waves stream M (8 per block).  Y stream: J = 64/K columns per tile, row
// splits while every thread still covers >= 1 row and the grid is short of
// ~4096 waves; row splits are whole multiples of 64 rows.  A single split
// makes the half one kernel that streams and solves (chosen for matrices of
// at most 2^18 entries, or by the caller).  NNLS kernels: one wave (64
// problems) per block up to k = 8, four waves beyond.
// fuse_x / fuse_y: 1 runs the half as one kernel whatever its splits, 0 as two
// kernels, -1 (automatic) as one kernel exactly when it has a single split.
Plan plan_shape(int64_t n, int64_t m, int64_t m_cap, int K, int x_splits = 0, int y_splits = 0, int fuse_x = -1,
                int fuse_y = -1) {
    Plan P;
    P.ldM = align_up((size_t)n, 32);
    P.ldX = align_up((size_t)n, 64);
    P.ldY = align_up((size_t)m_cap, 64);
    P.Tn = (int)ceil_div(n, nmfk::XTILE);
    int64_t sx = ceil_div(4096, (int64_t)P.Tn * nmfk::SWAVES);
    if (n * m <= (int64_t)1 << 18) sx = 1;   // small: stream and solve in one kernel per half
    if (x_splits > 0) sx = x_splits;
    sx = std::max<int64_t>(1, std::min<int64_t>(sx, std::min<int64_t>(kSxMax, m)));
    P.xcols = (int)ceil_div(m, sx);
    P.Sx = (int)ceil_div(m, P.xcols);
    P.J = nmfk::yhalf_cols(K);
    P.Tm = (int)ceil_div(m, P.J);
    int64_t sy = std::min<int64_t>(ceil_div(4096, (int64_t)P.Tm * nmfk::SWAVES), n / nmfk::STHR);
    if (n * m <= (int64_t)1 << 18) sy = 1;
    if (y_splits > 0) sy = y_splits;
    sy = std::max<int64_t>(1, std::min<int64_t>(sy, std::min<int64_t>(kSyMax, n)));
    // row splits are whole multiples of 64 rows (the Y stream loads row pairs
    // and needs even split starts), so Sy can come out below the request
    P.yrows = (int)(ceil_div(ceil_div(n, sy), 64) * 64);
    P.Sy = (int)ceil_div(n, P.yrows);
    P.Bx = (int)ceil_div(n, nmfk::NTHR);
    P.By = (int)ceil_div(m, nmfk::NTHR);
    P.Nx = (int)ceil_div(n, nmfk::nnls_threads(K));
    P.Ny = (int)ceil_div(m, nmfk::nnls_threads(K));
    P.Wx = (int)ceil_div(n, nmfk::WTHR);
    P.Wy = (int)ceil_div(m, nmfk::WTHR);
    P.FX = fuse_x < 0 ? P.Sx == 1 : fuse_x != 0;
    P.FY = fuse_y < 0 ? P.Sy == 1 : fuse_y != 0;
    return P;
}

struct Carve {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        const size_t at = align_up(off, 256);
        off = at + count * sizeof(T);
        return at;
    }
};

struct Offsets {
    size_t M, Mlo, X, Y, xmask, ymask, bx, by, gx, gy, xst, yst, cntf, tcnt, status, red, io, bad;
    size_t gpres, gslot, gmask, gcount, gtab;   // tables of the grouped first solves
    size_t ipm_base, total;
};

// Slots of the grouped-solve table: every passive set for small K, else
// the first 2048 distinct sets of a half (later ones take the plain loop).
constexpr int64_t group_slots(int K) { return K <= 11 ? (int64_t)1 << K : 2048; }

Offsets layout(int64_t n, int64_t m_cap, int K, const nmf_options &o) {
    const Plan P = plan_shape(n, m_cap, m_cap, K, o.x_splits, o.y_splits);
    const int64_t ByMax = ceil_div(m_cap, nmfk::NTHR);
    Offsets L;
    Carve c;
    L.M = c.take<double>((size_t)P.ldM * m_cap);
    L.Mlo = c.take<uint32_t>(o.gram_precision != NMF_GRAM_FP64 ? (size_t)P.ldM * m_cap : 0);
    L.X = c.take<double>((size_t)K * P.ldX);
    L.Y = c.take<double>((size_t)K * P.ldY);
    L.xmask = c.take<uint32_t>(P.ldX);
    L.ymask = c.take<uint32_t>(P.ldY);
    L.bx = c.take<double>((size_t)kSxMax * K * P.ldX);
    L.by = c.take<double>((size_t)kSyMax * K * P.ldY);   // Sy varies with m; <= kSyMax
    // statistics / Gram records: one per NNLS block, or one per stream tile
    // when a half runs as one kernel (Tn >= Bx rows, Tm >= By columns)
    const int64_t TmMax = ceil_div(m_cap, nmfk::yhalf_cols(K));
    const int64_t NyMax = ceil_div(m_cap, nmfk::WTHR);
    const int64_t RxMax = std::max<int64_t>(P.Wx, P.Tn),
                  RyMax = std::max<int64_t>(std::max<int64_t>(ByMax, NyMax), TmMax);
    L.gx = c.take<double>((size_t)RxMax * K * K);
    L.gy = c.take<double>((size_t)RyMax * K * K);
    L.xst = c.take<double>((size_t)RxMax * nmfk::NST);
    L.yst = c.take<double>((size_t)RyMax * nmfk::NST);
    L.cntf = c.take<unsigned>(4);
    L.tcnt = c.take<unsigned>((size_t)P.Tn + TmMax);   // tile arrivals of the one-kernel halves
    L.status = c.take<DevStatus>(1);
    L.red = c.take<double>(2 * kRedBlocks);
    L.io = c.take<double>((size_t)K * (n + m_cap));
    L.bad = c.take<unsigned>(4);
    const int64_t gcap = group_slots(K);
    L.gpres = c.take<uint8_t>((size_t)1 << K);
    L.gslot = c.take<int>((size_t)1 << K);
    L.gmask = c.take<uint32_t>((size_t)gcap);
    L.gcount = c.take<int>(1);
    L.gtab = c.take<double>((size_t)gcap * K * K);
    L.ipm_base = align_up(c.off, 256);
    size_t ipm = o.with_ipm ? nmfk::ipm_workspace_bytes(n, m_cap, K) : 0;
    L.total = L.ipm_base + ipm;
    return L;
}

}  // namespace

struct nmf_ctx {
    int64_t n = 0, m = 0, m_cap = 0;
    int K = 0;
    nmf_options opt;
    hipStream_t stream = nullptr;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    Offsets off;
    Plan plan;
    AnlsParams p;
    double *red = nullptr, *io = nullptr;
    unsigned *bad = nullptr;
    int stage = 1;
    int fuse_x = -1, fuse_y = -1;   // nmf_set_launch_fusion
    int grouped = 0;                // nmf_set_nnls_grouping
    double mnorm2 = 0.0;
    double ms1 = 0.0, ms2 = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DevStatus *hstat = nullptr;   // pinned host copy of the device status (read back after sweeps)
    DevStatus last1;   // stage-1 status at the hand-over to stage 2
    nmfk::IpmState ipm;
    std::string err;
};

static nmf_status fail(nmf_ctx *c, nmf_status st, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return st;
}

static nmf_status hip_fail(nmf_ctx *c, hipError_t e, const char *what) {
    return fail(c, NMF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, call)                                   \
    do {                                                  \
        hipError_t _e = (call);                           \
        if (_e != hipSuccess) return hip_fail(c, _e, #call); \
    } while (0)

static void refresh_shape(nmf_ctx *c) {
    // the grouped first solves run in the separate solve kernels
    c->plan = plan_shape(c->n, c->m, c->m_cap, c->K, c->opt.x_splits, c->opt.y_splits, c->grouped ? 0 : c->fuse_x,
                         c->grouped ? 0 : c->fuse_y);
    AnlsParams &p = c->p;
    p.n = c->n;
    p.m = c->m;
    p.Sx = c->plan.Sx;
    p.Tn = c->plan.Tn;
    p.xcols = c->plan.xcols;
    p.Sy = c->plan.Sy;
    p.Tm = c->plan.Tm;
    p.yrows = c->plan.yrows;
    p.Bx = c->plan.Bx;
    p.By = c->plan.By;
    p.Nx = c->plan.Nx;
    p.Ny = c->plan.Ny;
    p.Wx = c->plan.Wx;
    p.Wy = c->plan.Wy;
    p.fx = c->plan.FX ? 1 : 0;
    p.fy = c->plan.FY ? 1 : 0;
    p.Rx = p.fx ? p.Tn : p.Wx;
    p.Ry = p.fy ? p.Tm : p.Wy;
}

extern "C" {

void nmf_default_options(nmf_options *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->eps_tol = 1e-6;
    o->eps_stol = 1e-6;
    o->tau = 0.9;
    o->eta = 0.5;
    o->sigma_c = 0.01;
    o->rho0_factor = 1e-6;
    o->rho = 1e-6;
    o->inner_cap = 3;
    o->exact_hessian_switch = 1;
    o->max_anls_sweeps = 5000;
    o->max_ipm_iters = 1000;
    o->max_backtracks = 60;
    o->check_every = 32;
    o->gram_precision = NMF_GRAM_FP64;
    o->with_ipm = 1;
    o->seed = 0;
}

size_t nmf_workspace_bytes(int64_t n, int64_t m_capacity, int32_t k, const nmf_options *opts) {
    if (n < 1 || m_capacity < 1 || k < 1 || k > nmfk::KMAX) return 0;
    nmf_options o;
    if (opts) o = *opts;
    else nmf_default_options(&o);
    return layout(n, m_capacity, k, o).total;
}

const char *nmf_status_string(nmf_status s) {
    switch (s) {
        case NMF_OK: return "NMF_OK";
        case NMF_CONVERGED: return "NMF_CONVERGED";
        case NMF_EINVAL: return "NMF_EINVAL";
        case NMF_ENOMEM: return "NMF_ENOMEM";
        case NMF_EDEVICE: return "NMF_EDEVICE";
        case NMF_ENOTCONV: return "NMF_ENOTCONV";
        case NMF_ESINGULAR: return "NMF_ESINGULAR";
        case NMF_ESTATE: return "NMF_ESTATE";
        case NMF_ECAPACITY: return "NMF_ECAPACITY";
    }
    return "unknown";
}

const char *nmf_last_error(const nmf_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

nmf_status nmf_get_shape(const nmf_ctx *c, int64_t *n, int64_t *m, int32_t *k) {
    if (!c) return NMF_EINVAL;
    if (n) *n = c->n;
    if (m) *m = c->m;
    if (k) *k = c->K;
    return NMF_OK;
}

// Host draw of the seeded start (splitmix64 -> U(0,1)), scaled so that
// ||X0 Y0||_F = ||M||_F.
static double host_u01(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (idx + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

nmf_status nmf_create(const double *M, int64_t n, int64_t m, int64_t ldm, int32_t k, int64_t m_capacity,
                      const double *X0, const double *Y0, const nmf_options *opts, void *device_workspace,
                      size_t ws_bytes, void *hip_stream, nmf_ctx **out) {
    if (!out) return fail(nullptr, NMF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!M) return fail(nullptr, NMF_EINVAL, "M is NULL");
    if (n < 1 || m < 1 || k < 1 || k > nmfk::KMAX)
        return fail(nullptr, NMF_EINVAL, "need n >= 1, m >= 1, 1 <= k <= 16");
    if (m_capacity < m) return fail(nullptr, NMF_EINVAL, "m_capacity < m");
    if (ldm < n) return fail(nullptr, NMF_EINVAL, "ldm < n");
    if ((X0 == nullptr) != (Y0 == nullptr)) return fail(nullptr, NMF_EINVAL, "give both X0 and Y0 or neither");
    nmf_options o;
    if (opts) o = *opts;
    else nmf_default_options(&o);
    if (o.inner_cap < 1 || o.check_every < 1 || !(o.tau > 0 && o.tau < 1) || !(o.eta > 0 && o.eta < 1) ||
        o.x_splits < 0 || o.x_splits > kSxMax || o.y_splits < 0 || o.y_splits > kSyMax)
        return fail(nullptr, NMF_EINVAL, "invalid options");
    if (o.gram_precision < NMF_GRAM_FP64 || o.gram_precision > NMF_GRAM_BF16X2)
        return fail(nullptr, NMF_EINVAL, "unknown gram_precision");
    const Offsets L = layout(n, m_capacity, k, o);
    if (!device_workspace || ws_bytes < L.total)
        return fail(nullptr, NMF_ENOMEM, "workspace smaller than nmf_workspace_bytes()");
    if (((uintptr_t)device_workspace) % 256 != 0) return fail(nullptr, NMF_EINVAL, "workspace not 256-byte aligned");

    nmf_ctx *c = new (std::nothrow) nmf_ctx();
    if (!c) return fail(nullptr, NMF_ENOMEM, "host allocation failed");
    c->n = n;
    c->m = m;
    c->m_cap = m_capacity;
    c->K = k;
    c->opt = o;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (uint8_t *)device_workspace;
    c->ws_bytes = ws_bytes;
    c->off = L;
    AnlsParams &p = c->p;
    memset(&p, 0, sizeof(p));
    uint8_t *w = c->ws;
    p.M = (const double *)(w + L.M);
    p.Mlo = (const uint32_t *)(w + L.Mlo);
    p.prec = o.gram_precision;
    p.X = (double *)(w + L.X);
    p.Y = (double *)(w + L.Y);
    p.xmask = (uint32_t *)(w + L.xmask);
    p.ymask = (uint32_t *)(w + L.ymask);
    p.bx_part = (double *)(w + L.bx);
    p.by_part = (double *)(w + L.by);
    p.gx_part = (double *)(w + L.gx);
    p.gy_part = (double *)(w + L.gy);
    p.xstat = (double *)(w + L.xst);
    p.ystat = (double *)(w + L.yst);
    p.cnt_fin = (unsigned *)(w + L.cntf);
    p.tile_cnt = (unsigned *)(w + L.tcnt);
    p.st = (DevStatus *)(w + L.status);
    p.gcap = (int)group_slots(k);
    p.gpresent = (uint8_t *)(w + L.gpres);
    p.gslot = (int *)(w + L.gslot);
    p.gmask = (uint32_t *)(w + L.gmask);
    p.gcount = (int *)(w + L.gcount);
    p.gtab = (double *)(w + L.gtab);
    c->red = (double *)(w + L.red);
    c->io = (double *)(w + L.io);
    c->bad = (unsigned *)(w + L.bad);
    refresh_shape(c);
    p.ldM = c->plan.ldM;
    p.ldX = c->plan.ldX;
    p.ldY = c->plan.ldY;

    nmf_status st = NMF_OK;
    auto bail = [&](nmf_status s) {
        g_create_error = c->err;
        if (c->ev0) (void)hipEventDestroy(c->ev0);
        if (c->ev1) (void)hipEventDestroy(c->ev1);
        delete c;
        return s;
    };
#define CHK(call)                                                  \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return bail(hip_fail(c, _e, #call)); \
    } while (0)

    hipStream_t s = c->stream;
    CHK(hipEventCreate(&c->ev0));
    CHK(hipEventCreate(&c->ev1));
    // small regions start at zero (counters must be zero before the first sweep)
    CHK(hipMemsetAsync(w + L.bx, 0, L.io - L.bx, s));
    CHK(hipMemsetAsync(w + L.X, 0, L.bx - L.X, s));
    CHK(hipMemsetAsync(w + L.gpres, 0, (size_t)1 << k, s));   // no passive set marked
    CHK(hipMemcpy2DAsync((void *)p.M, (size_t)p.ldM * 8, M, (size_t)ldm * 8, (size_t)n * 8, (size_t)m,
                         hipMemcpyDefault, s));
    CHK(nmfk::launch_check_finite(p.M, n, m, p.ldM, c->red, kRedBlocks, s));
    CHK(nmfk::launch_make_lowprec(p, 0, m, s));
    std::vector<double> red(2 * kRedBlocks);
    CHK(hipMemcpyAsync(red.data(), c->red, red.size() * 8, hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    double mn2 = 0.0, nbad = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) {
        mn2 += red[b];
        nbad += red[kRedBlocks + b];
    }
    if (nbad > 0) {
        c->err = "M has NaN or Inf entries";
        return bail(NMF_EINVAL);
    }
    c->mnorm2 = mn2;

    const double *sx = X0, *sy = Y0;
    std::vector<double> hx, hy;
    if (!X0) {
        hx.resize((size_t)n * k);
        hy.resize((size_t)k * m);
        for (size_t q = 0; q < hx.size(); ++q) hx[q] = host_u01(o.seed, q);
        for (size_t q = 0; q < hy.size(); ++q) hy[q] = host_u01(o.seed ^ 0x5851F42D4C957F2Dull, q);
        double p2 = 0.0;
        std::vector<double> row(m);
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t j = 0; j < m; ++j) {
                double v = 0.0;
                for (int a = 0; a < k; ++a) v += hx[i * k + a] * hy[(size_t)a * m + j];
                p2 += v * v;
            }
        }
        const double scale = (p2 > 0 && mn2 > 0) ? sqrt(sqrt(mn2 / p2)) : 1.0;
        for (auto &v : hx) v *= scale;
        for (auto &v : hy) v *= scale;
        sx = hx.data();
        sy = hy.data();
    }
    // stage through io: [X0 n*k][Y0 k*m]
    CHK(hipMemcpyAsync(c->io, sx, (size_t)n * k * 8, hipMemcpyDefault, s));
    CHK(hipMemcpyAsync(c->io + (size_t)n * k, sy, (size_t)k * m * 8, hipMemcpyDefault, s));
    CHK(hipMemsetAsync(c->bad, 0, 16, s));
    CHK(nmfk::launch_factor_in(k, c->io, c->io + (size_t)n * k, p, c->bad, s));
    unsigned hbad = 0;
    CHK(hipMemcpyAsync(&hbad, c->bad, 4, hipMemcpyDeviceToHost, s));
    CHK(nmfk::launch_gram_y_init(k, p, s));
    DevStatus ds;
    memset(&ds, 0, sizeof(ds));
    ds.eps_stol = o.eps_stol;
    ds.max_sweeps = o.max_anls_sweeps;
    ds.ey_g2 = ds.ey_c2 = -1.0;
    ds.ey_g2_prev = ds.ey_c2_prev = -1.0;
    ds.E_prev = ds.E_cur = -1.0;
    ds.f_direct = -1.0;
    CHK(hipMemcpyAsync(p.st, &ds, sizeof(ds), hipMemcpyHostToDevice, s));
    CHK(hipStreamSynchronize(s));
    if (hbad) {
        c->err = "X0/Y0 have negative, NaN or Inf entries";
        return bail(NMF_EINVAL);
    }
    if (o.with_ipm) {
        st = nmfk::ipm_bind(c->ipm, w + L.ipm_base, n, m_capacity, k);
        if (st != NMF_OK) {
            c->err = "stage-2 workspace binding failed";
            return bail(st);
        }
    }
    // small pinned read-back buffers (the host waits on these copies after
    // every batch of sweeps and twice per interior-point iteration); without
    // them the copies go through pageable memory
    if (hipHostMalloc((void **)&c->hstat, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
        c->hstat = nullptr;
        (void)hipGetLastError();
    }
    if (o.with_ipm &&
        hipHostMalloc((void **)&c->ipm.hsc, sizeof(nmfk::IpmScal), hipHostMallocDefault) != hipSuccess) {
        c->ipm.hsc = nullptr;
        (void)hipGetLastError();
    }
#undef CHK
    *out = c;
    return NMF_OK;
}

nmf_status nmf_destroy(nmf_ctx *c) {
    if (!c) return NMF_OK;
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->hstat) (void)hipHostFree(c->hstat);
    if (c->ipm.hsc) (void)hipHostFree(c->ipm.hsc);
    delete c;
    return NMF_OK;
}

static nmf_status read_status(nmf_ctx *c, DevStatus &ds) {
    DevStatus *dst = c->hstat ? c->hstat : &ds;
    HIPCHK(c, hipMemcpyAsync(dst, c->p.st, sizeof(ds), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (dst != &ds) ds = *dst;
    return NMF_OK;
}

static void fill_stage1(nmf_ctx *c, const DevStatus &ds, nmf_report *r) {
    r->stage = c->stage;
    r->sweeps = ds.sweeps;
    r->step_rel = sqrt(ds.step2) / (1.0 + sqrt(ds.norm2));
    r->E0 = ds.E_cur >= 0 ? ds.E_cur : ds.E_prev;
    r->nnls_solves = (int64_t)ds.solves;
    r->nnls_failed = (int64_t)ds.fails;
    r->mask_changes = (int64_t)ds.changes;
    r->f = ds.f_direct;
    r->ms_stage1 = c->ms1;
    r->ms_stage2 = c->ms2;
}

static nmf_status enqueue_sweeps(nmf_ctx *c, int sweeps) {
    AnlsParams p = c->p;
    p.mode = 0;
    for (int t = 0; t < sweeps; ++t) {
        HIPCHK(c, nmfk::launch_xhalf(c->K, p, c->stream));
        HIPCHK(c, nmfk::launch_yhalf(c->K, p, c->stream));
    }
    return NMF_OK;
}

nmf_status nmf_anls_step(nmf_ctx *c, int32_t sweeps, nmf_report *r) {
    if (!c) return NMF_EINVAL;
    if (sweeps < 0) return fail(c, NMF_EINVAL, "sweeps < 0");
    if (c->stage != 1) return fail(c, NMF_ESTATE, "stage 2 has started");
    if (r) HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    nmf_status st = enqueue_sweeps(c, sweeps);
    if (st != NMF_OK) return st;
    if (!r) return NMF_OK;
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    DevStatus ds;
    st = read_status(c, ds);
    if (st != NMF_OK) return st;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->ms1 += ms;
    memset(r, 0, sizeof(*r));
    fill_stage1(c, ds, r);
    return ds.converged ? NMF_CONVERGED : NMF_OK;
}

nmf_status nmf_anls_profile(nmf_ctx *c, int32_t sweeps, double *ms) {
    if (!c || !ms) return NMF_EINVAL;
    if (sweeps < 1) return fail(c, NMF_EINVAL, "sweeps < 1");
    if (c->stage != 1) return fail(c, NMF_ESTATE, "stage 2 has started");
    std::vector<hipEvent_t> ev(8 * (size_t)sweeps, nullptr);   // a pair around each kernel
    nmf_status st = NMF_OK;
    for (auto &e : ev) {
        if (hipEventCreate(&e) != hipSuccess) { st = fail(c, NMF_EDEVICE, "hipEventCreate failed"); break; }
    }
    AnlsParams p = c->p;
    p.mode = 0;
    // the events are recorded by each kernel's own dispatch (no extra packets)
    const bool live[4] = {true, p.fx == 0, true, p.fy == 0};
    for (int t = 0; st == NMF_OK && t < sweeps; ++t) {
        hipEvent_t *e = &ev[8 * (size_t)t];
        bool ok = nmfk::launch_xstream(c->K, p, c->stream, e[0], e[1]) == hipSuccess &&
                  nmfk::launch_xnnls(c->K, p, c->stream, e[2], e[3]) == hipSuccess &&
                  nmfk::launch_ystream(c->K, p, c->stream, e[4], e[5]) == hipSuccess &&
                  nmfk::launch_ynnls(c->K, p, c->stream, e[6], e[7]) == hipSuccess;
        if (!ok) st = fail(c, NMF_EDEVICE, "launch failed");
    }
    double sum[4] = {0, 0, 0, 0};
    if (st == NMF_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = fail(c, NMF_EDEVICE, "sync failed");
    for (int t = 0; st == NMF_OK && t < sweeps; ++t) {
        for (int k = 0; k < 4; ++k) {
            if (!live[k]) continue;
            float a = 0.f;
            if (hipEventElapsedTime(&a, ev[8 * (size_t)t + 2 * k], ev[8 * (size_t)t + 2 * k + 1]) != hipSuccess) {
                st = fail(c, NMF_EDEVICE, "hipEventElapsedTime failed");
                break;
            }
            sum[k] += a;
        }
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st != NMF_OK) return st;
    for (int k = 0; k < 4; ++k) ms[k] = sum[k] / sweeps;
    return NMF_OK;
}

// E(.;0) of the current stage-1 iterate (measure-mode X-half) and the direct
// objective; results land in the device status.
static nmf_status measure_stage1(nmf_ctx *c) {
    AnlsParams p = c->p;
    p.mode = 1;
    p.prec = NMF_GRAM_FP64;   // the reported KKT error is always measured in FP64
    HIPCHK(c, nmfk::launch_xhalf(c->K, p, c->stream));
    HIPCHK(c, nmfk::launch_measure_finish(c->K, p, c->stream));
    HIPCHK(c, nmfk::launch_objective(c->K, p, c->red, kRedBlocks, c->stream));
    return NMF_OK;
}

nmf_status nmf_get_report(nmf_ctx *c, nmf_report *r) {
    if (!c || !r) return NMF_EINVAL;
    memset(r, 0, sizeof(*r));
    if (c->stage == 2) {
        nmfk::ipm_report(c->ipm, r, c->ms1, c->ms2);
        r->sweeps = c->last1.sweeps;
        r->nnls_solves = (int64_t)c->last1.solves;
        return NMF_OK;
    }
    nmf_status st = measure_stage1(c);
    if (st != NMF_OK) return st;
    DevStatus ds;
    st = read_status(c, ds);
    if (st != NMF_OK) return st;
    fill_stage1(c, ds, r);
    return NMF_OK;
}

nmf_status nmf_get_factors(nmf_ctx *c, double *X, double *Y) {
    if (!c) return NMF_EINVAL;
    if (c->stage == 2) {
        nmf_status st = nmfk::ipm_export(c->ipm, c->p, c->stream);
        if (st != NMF_OK) return fail(c, st, "stage-2 export failed");
    }
    HIPCHK(c, nmfk::launch_factor_out(c->K, c->p, c->io, c->io + (size_t)c->n * c->K, c->stream));
    if (X) HIPCHK(c, hipMemcpyAsync(X, c->io, (size_t)c->n * c->K * 8, hipMemcpyDefault, c->stream));
    if (Y)
        HIPCHK(c, hipMemcpyAsync(Y, c->io + (size_t)c->n * c->K, (size_t)c->K * c->m * 8, hipMemcpyDefault,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NMF_OK;
}

nmf_status nmf_get_masks(nmf_ctx *c, uint32_t *xm, uint32_t *ym) {
    if (!c) return NMF_EINVAL;
    if (xm) HIPCHK(c, hipMemcpyAsync(xm, c->p.xmask, (size_t)c->n * 4, hipMemcpyDefault, c->stream));
    if (ym) HIPCHK(c, hipMemcpyAsync(ym, c->p.ymask, (size_t)c->m * 4, hipMemcpyDefault, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NMF_OK;
}

nmf_status nmf_set_anls_budget(nmf_ctx *c, int32_t max_sweeps) {
    if (!c) return NMF_EINVAL;
    if (max_sweeps < 1) return fail(c, NMF_EINVAL, "max_sweeps < 1");
    if (c->stage != 1) return fail(c, NMF_ESTATE, "stage 2 has started");
    c->opt.max_anls_sweeps = max_sweeps;
    HIPCHK(c, nmfk::launch_rearm(c->p.st, max_sweeps, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NMF_OK;
}

nmf_status nmf_set_launch_shape(nmf_ctx *c, int32_t xs, int32_t ys) {
    if (!c) return NMF_EINVAL;
    if (xs < 0 || xs > kSxMax || ys < 0 || ys > kSyMax) return fail(c, NMF_EINVAL, "splits out of range");
    c->opt.x_splits = xs;
    c->opt.y_splits = ys;
    refresh_shape(c);
    if (c->stage == 1) {
        // the record layouts of the Gram partials follow the launch shape:
        // rebuild them from the current factors
        HIPCHK(c, nmfk::launch_gram_x_init(c->K, c->p, c->stream));
        HIPCHK(c, nmfk::launch_gram_y_init(c->K, c->p, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return NMF_OK;
}

nmf_status nmf_set_launch_fusion(nmf_ctx *c, int32_t fuse_x, int32_t fuse_y) {
    if (!c) return NMF_EINVAL;
    if (fuse_x < -1 || fuse_x > 1 || fuse_y < -1 || fuse_y > 1) return fail(c, NMF_EINVAL, "fusion mode not -1, 0 or 1");
    c->fuse_x = fuse_x;
    c->fuse_y = fuse_y;
    refresh_shape(c);
    if (c->stage == 1) {
        // the Gram records follow the kernel split of each half: rebuild them
        HIPCHK(c, nmfk::launch_gram_x_init(c->K, c->p, c->stream));
        HIPCHK(c, nmfk::launch_gram_y_init(c->K, c->p, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return NMF_OK;
}

nmf_status nmf_set_ipm_precision(nmf_ctx *c, int32_t mixed, int32_t refine_steps) {
    if (!c) return NMF_EINVAL;
    if (mixed != 0 && mixed != 1) return fail(c, NMF_EINVAL, "ipm precision not 0 or 1");
    if (refine_steps < 0 || refine_steps > 16) return fail(c, NMF_EINVAL, "refinement steps not in 0..16");
    if (!c->opt.with_ipm) return fail(c, NMF_ESTATE, "context created without stage-2 workspace");
    c->ipm.mixed = mixed;
    c->ipm.refine = refine_steps;
    return NMF_OK;
}

nmf_status nmf_set_nnls_grouping(nmf_ctx *c, int32_t on) {
    if (!c) return NMF_EINVAL;
    if (on != 0 && on != 1) return fail(c, NMF_EINVAL, "grouping not 0 or 1");
    c->grouped = on;
    c->p.grouped = on;
    refresh_shape(c);
    if (c->stage == 1) {
        // the Gram records follow the kernel split of each half: rebuild them
        HIPCHK(c, nmfk::launch_gram_x_init(c->K, c->p, c->stream));
        HIPCHK(c, nmfk::launch_gram_y_init(c->K, c->p, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return NMF_OK;
}

nmf_status nmf_get_launch_shape(const nmf_ctx *c, int32_t *out4) {
    if (!c || !out4) return NMF_EINVAL;
    out4[0] = c->p.Sx;
    out4[1] = c->p.Sy;
    out4[2] = c->p.fx;
    out4[3] = c->p.fy;
    return NMF_OK;
}

nmf_status nmf_get_duals(nmf_ctx *c, double *R, double *S) {
    if (!c) return NMF_EINVAL;
    if (c->stage != 2) return fail(c, NMF_ESTATE, "duals exist in stage 2 only");
    nmf_status st = nmfk::ipm_get_duals(c->ipm, c->p, R, S, c->stream);
    return st == NMF_OK ? NMF_OK : fail(c, st, "dual export failed");
}

nmf_status nmf_append_columns(nmf_ctx *c, const double *Mnew, int64_t mnew, int64_t ldm) {
    if (!c) return NMF_EINVAL;
    if (mnew < 0 || (mnew > 0 && !Mnew)) return fail(c, NMF_EINVAL, "bad new columns");
    if (mnew == 0) return NMF_OK;
    if (ldm < c->n) return fail(c, NMF_EINVAL, "ldm < n");
    if (c->m + mnew > c->m_cap) return fail(c, NMF_ECAPACITY, "m_capacity exceeded");
    hipStream_t s = c->stream;
    double *dst = (double *)c->p.M + (size_t)c->p.ldM * c->m;
    HIPCHK(c, hipMemcpy2DAsync(dst, (size_t)c->p.ldM * 8, Mnew, (size_t)ldm * 8, (size_t)c->n * 8,
                               (size_t)mnew, hipMemcpyDefault, s));
    HIPCHK(c, nmfk::launch_check_finite(dst, c->n, mnew, c->p.ldM, c->red, kRedBlocks, s));
    std::vector<double> red(2 * kRedBlocks);
    HIPCHK(c, hipMemcpyAsync(red.data(), c->red, red.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double add = 0.0, nbad = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) {
        add += red[b];
        nbad += red[kRedBlocks + b];
    }
    if (nbad > 0) return fail(c, NMF_EINVAL, "new columns have NaN or Inf entries");
    if (c->stage == 2) {
        nmf_status st = nmfk::ipm_export(c->ipm, c->p, s);
        if (st != NMF_OK) return fail(c, st, "stage-2 export failed");
        c->stage = 1;
    }
    const int64_t m_old = c->m;
    c->mnorm2 += add;
    HIPCHK(c, nmfk::launch_make_lowprec(c->p, m_old, m_old + mnew, s));
    HIPCHK(c, nmfk::launch_copy_columns_warm(c->K, c->p, m_old - 1, m_old, m_old + mnew, s));
    c->m = m_old + mnew;
    refresh_shape(c);
    // the Y-half over all columns: the new ones start from their neighbour
    HIPCHK(c, nmfk::launch_gram_x_init(c->K, c->p, s));
    AnlsParams p = c->p;
    p.mode = 2;
    HIPCHK(c, nmfk::launch_yhalf(c->K, p, s));
    // the stop rule must be re-earned on the grown problem, with a fresh budget
    HIPCHK(c, nmfk::launch_rearm(c->p.st, c->opt.max_anls_sweeps, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return NMF_OK;
}

nmf_status nmf_ipm_step(nmf_ctx *c, int32_t iters, nmf_report *r) {
    if (!c) return NMF_EINVAL;
    if (!c->opt.with_ipm) return fail(c, NMF_ESTATE, "context created without stage-2 workspace");
    if (iters < 0) return fail(c, NMF_EINVAL, "iters < 0");
    if (c->stage == 1) {
        nmf_status rs = read_status(c, c->last1);
        if (rs != NMF_OK) return rs;
        nmf_status st = nmfk::ipm_transition(c->ipm, c->p, c->opt, c->stream);
        if (st != NMF_OK) return fail(c, st, nmfk::ipm_last_error(c->ipm));
        c->stage = 2;
    }
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    nmf_status st = nmfk::ipm_iterate(c->ipm, c->p, c->opt, iters, c->stream);
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->ms2 += ms;
    if (st != NMF_OK && st != NMF_CONVERGED && st != NMF_ENOTCONV)
        return fail(c, st, nmfk::ipm_last_error(c->ipm));
    if (r) {
        memset(r, 0, sizeof(*r));
        nmf_status rs = nmfk::ipm_report(c->ipm, r, c->ms1, c->ms2);
        if (rs != NMF_OK) return fail(c, rs, "report failed");
        r->sweeps = c->last1.sweeps;
        r->nnls_solves = (int64_t)c->last1.solves;
        r->nnls_failed = (int64_t)c->last1.fails;
        r->mask_changes = (int64_t)c->last1.changes;
        r->step_rel = sqrt(c->last1.step2) / (1.0 + sqrt(c->last1.norm2));
    }
    return st;
}

nmf_status nmf_ipm_profile(nmf_ctx *c, int32_t iters, double *ms, int64_t *counts) {
    if (!c || !ms) return NMF_EINVAL;
    nmfk::IpmState &s = c->ipm;
    if (!c->opt.with_ipm) return fail(c, NMF_ESTATE, "context created without stage-2 workspace");
    for (int q = 0; q < 4; ++q) {
        s.prof_ms[q] = 0.0;
        s.prof_n[q] = 0;
    }
    if (hipEventCreate(&s.pev[0]) != hipSuccess || hipEventCreate(&s.pev[1]) != hipSuccess) {
        if (s.pev[0]) (void)hipEventDestroy(s.pev[0]);
        s.pev[0] = s.pev[1] = nullptr;
        return fail(c, NMF_EDEVICE, "hipEventCreate failed");
    }
    s.prof = true;
    const int64_t it0 = s.iters;
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    const nmf_status st = nmf_ipm_step(c, iters, nullptr);
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev1));
    float total = 0.f;
    (void)hipEventElapsedTime(&total, c->ev0, c->ev1);
    s.prof = false;
    (void)hipEventDestroy(s.pev[0]);
    (void)hipEventDestroy(s.pev[1]);
    s.pev[0] = s.pev[1] = nullptr;
    const int64_t done = s.iters - it0;
    for (int q = 0; q < 4; ++q) ms[q] = s.prof_n[q] ? s.prof_ms[q] / (double)s.prof_n[q] : 0.0;
    ms[4] = done > 0 ? total / (double)done : 0.0;
    if (counts) {
        for (int q = 0; q < 4; ++q) counts[q] = s.prof_n[q];
        counts[4] = done;
    }
    return st;
}

nmf_status nmf_solve(nmf_ctx *c, nmf_report *r) {
    if (!c) return NMF_EINVAL;
    nmf_status st = NMF_OK;
    if (c->stage == 1) {
        DevStatus ds;
        HIPCHK(c, hipEventRecord(c->ev0, c->stream));
        for (;;) {
            st = enqueue_sweeps(c, c->opt.check_every);
            if (st != NMF_OK) return st;
            st = read_status(c, ds);
            if (st != NMF_OK) return st;
            if (ds.converged) break;
        }
        HIPCHK(c, hipEventRecord(c->ev1, c->stream));
        HIPCHK(c, hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        c->ms1 += ms;
        if (!c->opt.with_ipm) {
            if (r) return nmf_get_report(c, r);
            return NMF_OK;
        }
    }
    st = nmf_ipm_step(c, c->opt.max_ipm_iters, r);
    return st;
}

// ------------------------------------------------------------------ batches
struct nmf_batch {
    struct Group {
        int K = 0, prec = 0;
        std::vector<int> members;
        nmfk::BatchGroup g;
    };
    std::vector<nmf_ctx *> ctxs;
    std::vector<Group> groups;
    hipStream_t stream = nullptr;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_sweeps = 0;
    std::vector<int> order;       // table position -> index in ctxs
    long long *poll = nullptr;    // device: [count][2] converged, sweeps
    // K-groups are independent problems: with side streams, each group's
    // sweeps run on a stream of their own, forked from and joined back to
    // `stream` by events (also inside a captured graph, as parallel branches)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;   // [0]: fork, [1 + s]: join of side stream s
    std::string err;
};

static void drop_side_streams(nmf_batch *b) {
    for (hipStream_t s : b->side) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    b->side.clear();
    b->ev.clear();
}

// One side stream per K-group, at most kMaxSideStreams (default priority).
constexpr int kMaxSideStreams = 8;
static hipError_t make_side_streams(nmf_batch *b) {
    const int ns = std::min((int)b->groups.size(), kMaxSideStreams);
    if (ns < 2) return hipSuccess;
    for (int q = 0; q <= ns; ++q) {
        hipEvent_t e = nullptr;
        const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        b->ev.push_back(e);
    }
    for (int q = 0; q < ns; ++q) {
        hipStream_t st = nullptr;
        const hipError_t r = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (r != hipSuccess) return r;
        b->side.push_back(st);
    }
    return hipSuccess;
}

// Offset tables: NBK arrays of (members + 1) entries per group, at most
// NBK * 2 * count entries over all groups (a group has at least one member).
static size_t offsets_bytes(size_t count) { return align_up((size_t)nmfk::NBK * 2 * count * sizeof(int), 256); }

static constexpr size_t batch_bytes(int32_t count) {
    return ((size_t)count * sizeof(AnlsParams) + 255) / 256 * 256 +
           ((size_t)nmfk::NBK * 2 * count * sizeof(int) + 255) / 256 * 256 +
           ((size_t)2 * count * sizeof(long long) + 255) / 256 * 256 + 256;
}

// Batch tables of nmf_batch_create_static: one copy per device, in device
// memory that the library owns for the life of the process.  Host code never
// passes the array's name to a kernel or a copy: it uses the address
// hipGetSymbolAddress returns on each device (static_scratch()).
constexpr size_t kStaticBatchBytes = batch_bytes(NMF_BATCH_STATIC_MAX);
static __device__ __align__(256) uint8_t scratch[kStaticBatchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
static hipError_t static_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

static void drop_graph(nmf_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_sweeps = 0;
}

size_t nmf_batch_workspace_bytes(int32_t count) { return count < 1 ? 0 : batch_bytes(count); }

nmf_status nmf_batch_refresh(nmf_batch *b) {
    if (!b) return NMF_EINVAL;
    drop_graph(b);
    b->groups.clear();
    for (int q = 0; q < (int)b->ctxs.size(); ++q) {
        nmf_ctx *c = b->ctxs[q];
        if (c->stage != 1) {
            b->err = "every context of a batch must be in stage 1";
            return NMF_ESTATE;
        }
        int gi = -1;
        for (int t = 0; t < (int)b->groups.size(); ++t)
            if (b->groups[t].K == c->K && b->groups[t].prec == c->opt.gram_precision) gi = t;
        if (gi < 0) {
            b->groups.emplace_back();
            b->groups.back().K = c->K;
            b->groups.back().prec = c->opt.gram_precision;
            gi = (int)b->groups.size() - 1;
        }
        b->groups[gi].members.push_back(q);
    }
    // tables: all groups' AnlsParams back to back, then their offsets
    std::vector<AnlsParams> tab;
    std::vector<int> offs;
    const size_t count = b->ctxs.size();
    AnlsParams *dtab = (AnlsParams *)b->ws;
    int *doff = (int *)(b->ws + align_up(count * sizeof(AnlsParams), 256));
    b->poll = (long long *)(b->ws + align_up(count * sizeof(AnlsParams), 256) + offsets_bytes(count));
    b->order.clear();
    for (auto &g : b->groups) {
        const int np = (int)g.members.size();
        g.g.table = dtab + tab.size();
        g.g.off = doff + offs.size();
        g.g.count = np;
        std::vector<int> o[nmfk::NBK];
        for (auto &v : o) v.assign(1, 0);
        for (int q : g.members) {
            AnlsParams p = b->ctxs[q]->p;
            p.mode = 0;
            p.grouped = 0;   // the batched sweeps build no grouping tables
            tab.push_back(p);
            b->order.push_back(q);
            g.g.single = p;
            const bool fx = p.fx != 0, fy = p.fy != 0;
            const int cnt[nmfk::NBK] = {fx ? 0 : p.Tn * p.Sx, fx ? 0 : p.Nx, fy ? 0 : p.Tm * p.Sy,
                                        fy ? 0 : p.Ny,     fx ? p.Tn * p.Sx : 0, fy ? p.Tm * p.Sy : 0};
            for (int k = 0; k < nmfk::NBK; ++k) o[k].push_back(o[k].back() + cnt[k]);
        }
        for (int k = 0; k < nmfk::NBK; ++k) {
            g.g.blocks[k] = o[k].back();
            offs.insert(offs.end(), o[k].begin(), o[k].end());
        }
    }
    if (offs.size() * sizeof(int) > offsets_bytes(count)) {
        b->err = "batch offset tables exceed their workspace region";
        return NMF_ENOMEM;
    }
    if (hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(AnlsParams), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipMemcpyAsync(doff, offs.data(), offs.size() * sizeof(int), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = "table upload failed";
        return NMF_EDEVICE;
    }
    return NMF_OK;
}

static nmf_status batch_create(nmf_ctx *const *ctxs, int32_t count, void *ws, size_t ws_bytes, void *stream,
                               bool concurrent, nmf_batch **out) {
    if (!out || !ctxs || count < 1) return fail(nullptr, NMF_EINVAL, "bad batch arguments");
    *out = nullptr;
    if (!ws || ws_bytes < batch_bytes(count)) return fail(nullptr, NMF_ENOMEM, "batch workspace too small");
    if (((uintptr_t)ws) % 256 != 0) return fail(nullptr, NMF_EINVAL, "batch workspace not 256-byte aligned");
    nmf_batch *b = new (std::nothrow) nmf_batch();
    if (!b) return fail(nullptr, NMF_ENOMEM, "host allocation failed");
    for (int q = 0; q < count; ++q) {
        if (!ctxs[q]) {
            delete b;
            return fail(nullptr, NMF_EINVAL, "NULL context in batch");
        }
        b->ctxs.push_back(ctxs[q]);
    }
    b->stream = (hipStream_t)stream;
    b->ws = (uint8_t *)ws;
    b->ws_bytes = ws_bytes;
    nmf_status st = nmf_batch_refresh(b);
    if (st != NMF_OK) {
        g_create_error = b->err;
        delete b;
        return st;
    }
    if (concurrent) {
        const hipError_t e = make_side_streams(b);
        if (e != hipSuccess) {
            drop_side_streams(b);
            delete b;
            return hip_fail(nullptr, e, "side streams of the batch");
        }
    }
    *out = b;
    return NMF_OK;
}

nmf_status nmf_batch_create(nmf_ctx *const *ctxs, int32_t count, void *ws, size_t ws_bytes, void *stream,
                            nmf_batch **out) {
    return batch_create(ctxs, count, ws, ws_bytes, stream, true, out);
}

nmf_status nmf_batch_create_static(nmf_ctx *const *ctxs, int32_t count, void *stream, nmf_batch **out) {
    if (!out || !ctxs || count < 1) return fail(nullptr, NMF_EINVAL, "bad batch arguments");
    *out = nullptr;
    if (count > NMF_BATCH_STATIC_MAX)
        return fail(nullptr, NMF_ECAPACITY,
                    "nmf_batch_create_static: " + std::to_string(count) + " contexts exceed the static batch limit of " +
                        std::to_string(NMF_BATCH_STATIC_MAX));
    void *ws = nullptr;
    const hipError_t e = static_scratch(&ws);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress of the static batch tables");
    return batch_create(ctxs, count, ws, kStaticBatchBytes, stream, false, out);
}

static nmf_status batch_enqueue(nmf_batch *b, int sweeps) {
    const int ns = (int)b->side.size();
    if (ns == 0) {
        for (int t = 0; t < sweeps; ++t)
            for (auto &g : b->groups)
                if (nmfk::launch_batch_sweep(g.K, g.prec, g.g, b->stream) != hipSuccess) {
                    b->err = "batched launch failed";
                    return NMF_EDEVICE;
                }
        return NMF_OK;
    }
    if (hipEventRecord(b->ev[0], b->stream) != hipSuccess) {
        b->err = "batch fork event failed";
        return NMF_EDEVICE;
    }
    for (int q = 0; q < ns; ++q)
        if (hipStreamWaitEvent(b->side[q], b->ev[0], 0) != hipSuccess) {
            b->err = "batch fork wait failed";
            return NMF_EDEVICE;
        }
    for (int t = 0; t < sweeps; ++t)
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            auto &g = b->groups[gi];
            if (nmfk::launch_batch_sweep(g.K, g.prec, g.g, b->side[gi % ns]) != hipSuccess) {
                b->err = "batched launch failed";
                return NMF_EDEVICE;
            }
        }
    for (int q = 0; q < ns; ++q)
        if (hipEventRecord(b->ev[1 + q], b->side[q]) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->ev[1 + q], 0) != hipSuccess) {
            b->err = "batch join failed";
            return NMF_EDEVICE;
        }
    return NMF_OK;
}

nmf_status nmf_batch_anls_step(nmf_batch *b, int32_t sweeps, int32_t use_graph) {
    if (!b || sweeps < 0) return NMF_EINVAL;
    if (sweeps == 0) return NMF_OK;
    if (!use_graph) return batch_enqueue(b, sweeps);
    if (!b->exec || b->graph_sweeps != sweeps) {
        drop_graph(b);
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            b->err = "stream capture failed (the batch stream must not be the default stream)";
            return NMF_EDEVICE;
        }
        nmf_status st = batch_enqueue(b, sweeps);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (st != NMF_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            b->err = "graph capture failed";
            return NMF_EDEVICE;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            b->err = "graph instantiation failed";
            return NMF_EDEVICE;
        }
        b->graph_sweeps = sweeps;
    }
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) {
        b->err = "graph launch failed";
        return NMF_EDEVICE;
    }
    return NMF_OK;
}

nmf_status nmf_batch_poll(nmf_batch *b, int32_t *converged, int64_t *sweeps) {
    if (!b) return NMF_EINVAL;
    const int count = (int)b->ctxs.size();
    std::vector<long long> h(2 * (size_t)count);
    if (nmfk::launch_batch_poll((const AnlsParams *)b->ws, count, b->poll, b->stream) != hipSuccess ||
        hipMemcpyAsync(h.data(), b->poll, h.size() * sizeof(long long), hipMemcpyDeviceToHost, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = "status poll failed";
        return NMF_EDEVICE;
    }
    for (int t = 0; t < count; ++t) {
        const int q = b->order[t];
        if (converged) converged[q] = (int32_t)h[2 * (size_t)t];
        if (sweeps) sweeps[q] = (int64_t)h[2 * (size_t)t + 1];
    }
    return NMF_OK;
}

nmf_status nmf_batch_sync(nmf_batch *b) {
    if (!b) return NMF_EINVAL;
    return hipStreamSynchronize(b->stream) == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

nmf_status nmf_batch_destroy(nmf_batch *b) {
    if (!b) return NMF_OK;
    drop_graph(b);
    drop_side_streams(b);
    delete b;
    return NMF_OK;
}

}  // extern "C"
