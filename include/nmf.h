/*
 * nmf.h - C ABI of the MI355X (gfx950) library for two-stage non-negative
 * matrix factorisation of streaming data, after Gu, Du and Billinge, "A fast
 * two-stage algorithm for non-negative matrix factorization in streaming data".
 *
 * Problem (eq. (1)): minimise f(X, Y) = 1/2 ||X Y - M||_F^2 subject to X >= 0,
 * Y >= 0, with M n x m, X n x k, Y k x m, n >> m >> k.
 *
 * Stage 1 (Sec. II, Alg. 1): alternating non-negative least squares, X-half
 * then Y-half; every row of X and every column of Y is one k-variable NNLS
 * problem, eq. (2), solved by the active-set method of Lawson and Hanson,
 * warm-started from the same row's (column's) previous solution and active set.
 * Stage 2 (Sec. III, IV, Alg. 2, Alg. 3): the transition eq. (21)-(25), then a
 * primal-dual line-search interior-point method whose Newton system eq. (12) is
 * solved through n k x k block Cholesky factors and an mk x mk Schur complement,
 * eq. (20).
 *
 * Conventions shared by every entry point
 *   - All functions return an nmf_status and never throw.  On failure
 *     nmf_last_error() describes the cause.
 *   - Memory: the library never allocates device memory.  The caller sizes a
 *     device workspace with nmf_workspace_bytes(), allocates it (for instance as
 *     a torch uint8 tensor) and lends it to nmf_create() until nmf_destroy().
 *     The context itself is a small host object owned by the library.
 *   - Pointers marked "host or device" may point to either; the library copies
 *     through unified addressing and takes no ownership.  Copies out of pageable
 *     host memory are synchronous.
 *   - Streams: all device work is enqueued on the hipStream_t given to
 *     nmf_create() (passed as void*, NULL = the default stream).  Functions that
 *     fill an nmf_report synchronise that stream; with report == NULL the step
 *     functions only enqueue work.
 *   - Layouts: M is column-major (element (i, j) at M[j*ldm + i], one time
 *     instant per column, ldm >= n); X is n x k row-major; Y is k x m
 *     row-major.  All values are IEEE double.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef NMF_H
#define NMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_ctx nmf_ctx;

typedef enum {
    NMF_OK = 0,
    NMF_CONVERGED = 1,      /* the requested stopping rule holds */
    NMF_EINVAL = -1,        /* bad argument: sizes, NULL pointers, NaN/Inf or negative entries */
    NMF_ENOMEM = -2,        /* workspace too small */
    NMF_EDEVICE = -3,       /* a HIP call failed */
    NMF_ENOTCONV = -4,      /* iteration cap reached; the iterate is valid and feasible */
    NMF_ESINGULAR = -5,     /* numerical breakdown of the Gauss-Newton Schur matrix */
    NMF_ESTATE = -6,        /* call not valid in the current stage */
    NMF_ECAPACITY = -7      /* nmf_append_columns beyond m_capacity */
} nmf_status;

/* Precision of the two Gram products M Y^T and X^T M that stream M (stage 1).
 * FP64 reads M as double.  FP32 and BF16X2 keep an extra reduced-precision copy
 * of M (4 bytes per entry: one float, or a bf16 high part and a bf16 low part)
 * and accumulate in FP32; the k x k solves and stage 2 stay FP64. */
typedef enum {
    NMF_GRAM_FP64 = 0,
    NMF_GRAM_FP32 = 1,
    NMF_GRAM_BF16X2 = 2
} nmf_gram_precision;

typedef struct {
    double eps_tol;        /* stop when E(.;0) <= eps_tol, eq. (10); Sec. V-A uses 1e-6 */
    double eps_stol;       /* stage-1 relative step tolerance, Sec. IV (default 1e-6) */
    double tau;            /* fraction to the boundary, eq. (7) (0.9) */
    double eta;            /* Armijo constant, Alg. 3 (0.5) */
    double sigma_c;        /* exact-Hessian switch threshold, Sec. IV (0.01) */
    double rho0_factor;    /* eq. (22) (1e-6) */
    double rho;            /* Hessian shift of eq. (11); eq. (25) sets it to the paper's eps_TOL (1e-6) */
    int32_t inner_cap;     /* interior-point iterations at one mu before the mu update (3) */
    int32_t exact_hessian_switch; /* 1: switch to the Hessian eq. (27) when sigma <= sigma_c */
    int32_t max_anls_sweeps;      /* stage-1 cap (5000) */
    int32_t max_ipm_iters;        /* stage-2 cap on inner iterations (1000) */
    int32_t max_backtracks;       /* Armijo halvings (60) */
    int32_t check_every;          /* stage-1 sweeps enqueued between host reads of the stop rule (32) */
    int32_t gram_precision;       /* nmf_gram_precision (NMF_GRAM_FP64) */
    int32_t with_ipm;             /* 1: reserve workspace for stage 2 (mk x mk Schur matrix) */
    int32_t x_splits;             /* stage-1 launch shape: column splits of the X-half (0 = automatic, <= 64) */
    int32_t y_splits;             /* stage-1 launch shape: row splits of the Y-half (0 = automatic, <= 64) */
    uint64_t seed;                /* initial point when X0/Y0 are NULL */
} nmf_options;

typedef struct {
    double f;              /* objective 1/2 ||XY - M||^2 at the current iterate (direct pass) */
    double E0;             /* E(.;0) at the current iterate (stage 1: r = max(graX,0), s = max(graY,0)) */
    double Emu;            /* E(.;mu) (stage 2) */
    double mu, sigma;      /* barrier parameter and last centring value (stage 2) */
    double step_rel;       /* last stage-1 step / (1 + ||(x, y)||) */
    int32_t stage;         /* 1 = ANLS, 2 = interior point */
    int32_t flag;          /* 1 while the exact Hessian eq. (27) is in use */
    int64_t sweeps;        /* stage-1 sweeps done */
    int64_t ipm_iters;     /* stage-2 inner iterations done */
    int64_t ipm_outer;     /* stage-2 mu updates done */
    int64_t backtracks;    /* Armijo halvings taken */
    int64_t nnls_solves;   /* k x k linear solves inside the active-set method */
    int64_t nnls_failed;   /* NNLS problems that hit their solve cap */
    int64_t mask_changes;  /* rows/columns whose active set changed in stage 1 */
    int64_t exact_steps;   /* stage-2 steps taken with the exact Hessian */
    int64_t fallbacks;     /* exact-Hessian steps rejected (non-descent or indefinite) */
    double ms_stage1, ms_stage2;  /* device time of the two stages (events) */
} nmf_report;

/* Fills *opts with the defaults listed above. */
void nmf_default_options(nmf_options *opts);

/* Bytes of device workspace nmf_create() needs for these sizes.  Returns 0 for
 * invalid sizes (n < 1, m_capacity < 1, k < 1 or k > 16). */
size_t nmf_workspace_bytes(int64_t n, int64_t m_capacity, int32_t k, const nmf_options *opts);

/* Builds a context: copies M (n x m, column-major, leading dimension ldm, host
 * or device) into the workspace, sets the initial point from X0 (n x k
 * row-major) and Y0 (k x m row-major), both host or device and >= 0, or from a
 * seeded U(0,1) draw scaled so that ||X0 Y0||_F = ||M||_F when both are NULL.
 * m_capacity >= m reserves room for columns appended later.  M must be finite
 * (entries may be negative).  opts may be NULL (defaults).  The workspace
 * (device, >= nmf_workspace_bytes, 256-byte aligned) stays borrowed until
 * nmf_destroy().  Errors: NMF_EINVAL, NMF_ENOMEM, NMF_EDEVICE. */
nmf_status nmf_create(const double *M, int64_t n, int64_t m, int64_t ldm, int32_t k,
                      int64_t m_capacity, const double *X0, const double *Y0,
                      const nmf_options *opts, void *device_workspace, size_t ws_bytes,
                      void *hip_stream, nmf_ctx **out);

/* Stage 1: enqueues `sweeps` ANLS sweeps (Alg. 1: X-half, then Y-half).  Once
 * the Sec. IV step rule holds the remaining enqueued sweeps do nothing.  With a
 * report the call synchronises and returns NMF_CONVERGED if the rule holds.
 * NMF_ESTATE once stage 2 has started. */
nmf_status nmf_anls_step(nmf_ctx *ctx, int32_t sweeps, nmf_report *report);

/* Stage 2: on the first call performs the transition eq. (21)-(25), then runs
 * up to `iters` inner iterations of Alg. 3 (with the mu updates between them).
 * Synchronises after every iteration (the Armijo search and the loop tests are
 * decided on the host from device-computed scalars).  Returns NMF_CONVERGED
 * when E(.;0) <= eps_tol. */
nmf_status nmf_ipm_step(nmf_ctx *ctx, int32_t iters, nmf_report *report);

/* Alg. 3 to the end: stage 1 to the step rule (or its cap), then stage 2 to
 * E(.;0) <= eps_tol.  Returns NMF_CONVERGED, or NMF_ENOTCONV at a cap. */
nmf_status nmf_solve(nmf_ctx *ctx, nmf_report *report);

/* Streaming: appends mnew columns (n x mnew, column-major, leading dimension
 * ldm, host or device) to M.  The new columns of Y are solved at once by the
 * NNLS of the Y-half, warm-started from the last existing column, and the
 * context returns to stage 1 (the duals of the grown problem are not known)
 * with a fresh budget of max_anls_sweeps sweeps for its stop rule.
 * NMF_ECAPACITY beyond m_capacity. */
nmf_status nmf_append_columns(nmf_ctx *ctx, const double *Mnew, int64_t mnew, int64_t ldm);

/* Copies the current factors out: X as n x k row-major and Y as k x m
 * row-major (host or device; either may be NULL).  Synchronises. */
nmf_status nmf_get_factors(nmf_ctx *ctx, double *X, double *Y);

/* Stage 2 only: copies the dual variables of eq. (3) at the current iterate,
 * R as n x k row-major (r = vec(R^T)) and S as k x m row-major (s = vec(S)),
 * host or device; either may be NULL.  NMF_ESTATE in stage 1. */
nmf_status nmf_get_duals(nmf_ctx *ctx, double *R, double *S);

/* Copies the stage-1 passive-set masks (bit a set when entry a is > 0) of the
 * n rows of X and the m columns of Y (host or device; either may be NULL). */
nmf_status nmf_get_masks(nmf_ctx *ctx, uint32_t *xmask, uint32_t *ymask);

/* Fills a report for the current iterate (direct objective pass, E(.;0)).
 * Synchronises. */
nmf_status nmf_get_report(nmf_ctx *ctx, nmf_report *report);

/* Profiling: enqueues `sweeps` stage-1 sweeps like nmf_anls_step() with HIP
 * events recorded by every kernel's own dispatch, synchronises, and writes
 * the mean device time in milliseconds of the four stage-1 steps to
 * ms[0..3]: the X-half stream (B_X = M Y^T), the row NNLS, the Y-half stream
 * (B_Y = X^T M) and the column NNLS.  A half with a single split is one
 * kernel: its time is in the stream entry and its NNLS entry is 0.  Sweeps
 * after the stop rule holds return at once and are still counted. */
nmf_status nmf_anls_profile(nmf_ctx *ctx, int32_t sweeps, double *ms);

/* Profiling of stage 2: runs like nmf_ipm_step(ctx, iters, NULL) while timing
 * the dense steps of the Newton solve of Sec. III-B with HIP events (each
 * timed region is synchronised, so the call runs slower than nmf_ipm_step).
 * ms[0..4] (host, caller-owned): mean device milliseconds of one Gauss-Newton
 * Schur formation (eq. (20)), one exact-Hessian formation (eq. (27)), one
 * Cholesky factorisation of the Schur matrix, one pair of triangular solves,
 * and the wall time per inner iteration of the whole call.  counts[0..4]
 * (host, may be NULL): how many of each were timed and inner iterations run.
 * Returns what nmf_ipm_step returns. */
nmf_status nmf_ipm_profile(nmf_ctx *ctx, int32_t iters, double *ms, int64_t *counts);

/* Re-plans the stage-1 launch shape of a context: column splits of the X-half
 * and row splits of the Y-half (0 = automatic, at most 64 each).  A single
 * split runs that half as one kernel that streams M and solves its tile.
 * Results do not change beyond the rounding of the split sums.  Synchronises
 * (the Gram partial sums are rebuilt for the new layout).  Used by the
 * autotuner. */
nmf_status nmf_set_launch_shape(nmf_ctx *ctx, int32_t x_splits, int32_t y_splits);

/* Chooses how each stage-1 half is launched (Alg. 1 runs the X-half, then the
 * Y-half): 1 = one kernel (every split of a tile streams its share of M; the
 * last split of the tile to finish, found by a per-tile counter, sums the
 * partials in split order and solves the tile's rows or columns), 0 = a
 * streaming kernel followed by an NNLS kernel, -1 = automatic (one kernel
 * exactly when the half has a single split; the default).  Results do not
 * change beyond the rounding of the sums.  Synchronises (the Gram partial
 * sums are rebuilt).  NMF_EINVAL for other values.  Used by the autotuner. */
nmf_status nmf_set_launch_fusion(nmf_ctx *ctx, int32_t fuse_x, int32_t fuse_y);

/* The stage-1 launch plan in effect: out4 = {x splits, y splits, X-half is one
 * kernel (0/1), Y-half is one kernel (0/1)}.  out4 is host memory owned by the
 * caller. */
nmf_status nmf_get_launch_shape(const nmf_ctx *ctx, int32_t *out4);

/* Passive-set grouping of the stage-1 NNLS problems (Sec. II cites the
 * grouping of right-hand sides that share a passive set, so that one
 * factorisation serves all of them).  on = 1: in every sweep each half first
 * forms (G_PP)^-1 once for every distinct warm-start passive set P of its
 * problems (at most 2048 sets for k >= 12; problems past that take the plain
 * loop), and each problem tries z = (G_PP)^-1 b, the first solve of its
 * warm-started Lawson-Hanson loop; it keeps z when z > 0 on P and the loop's
 * optimality test passes, and otherwise runs the loop from the same start.
 * The results are those of on = 0 up to the rounding of that solve.  The
 * halves then run as separate stream and solve kernels (no one-kernel
 * halves).  on = 0 (the default) restores the per-problem loop.  Errors:
 * NMF_EINVAL. */
nmf_status nmf_set_nnls_grouping(nmf_ctx *ctx, int32_t on);

/* Mixed-precision interior point (the dense Schur algebra is the cost that
 * Sec. III-B says grows with m).  mixed = 1: the exact-Hessian Schur
 * complement of eq. (27) is formed on FP32 matrix cores (its rank update
 * V^T V with V rounded to FP32; S is stored, factored and solved in FP64),
 * and every direction solved with that factor is refined refine_steps times
 * against the FP64 operator, d <- d + S~^-1 (rhs - S d), with S applied
 * without forming it.  The Gauss-Newton formation of eq. (20) stays FP64: its
 * cost is in vector-unit products, which FP32 does not speed up here.
 * mixed = 0 (the default): FP64 throughout.  Errors: NMF_EINVAL (mixed not 0
 * or 1, refine_steps not in 0..16), NMF_ESTATE (created with with_ipm = 0). */
nmf_status nmf_set_ipm_precision(nmf_ctx *ctx, int32_t mixed, int32_t refine_steps);

/* Sets the stage-1 sweep budget (options.max_anls_sweeps, >= 1) used from now
 * on, and re-arms the stop rule of Sec. IV: the next sweeps run until it holds
 * again or `max_sweeps` more sweeps are done.  Every later
 * nmf_append_columns() grants the same budget afresh.  For streaming callers
 * that bound the work of each arriving block of columns.  Stage 1 only
 * (NMF_ESTATE otherwise). */
nmf_status nmf_set_anls_budget(nmf_ctx *ctx, int32_t max_sweeps);

/* ------------------------------------------------------------------ batches
 * Many independent problems swept together (stage 1): the contexts of a batch
 * are grouped by (k, gram precision) and every group runs each of the four
 * stage-1 kernels as one flattened launch in which each block serves one
 * problem's block of its own launch shape.  A problem's results are bitwise
 * the ones its own nmf_anls_step() would give; problems that meet their stop
 * rule idle.  For callers that sweep many small problems at once. */
typedef struct nmf_batch nmf_batch;

/* Device workspace a batch of `count` contexts needs (tables and offsets). */
size_t nmf_batch_workspace_bytes(int32_t count);

/* Builds a batch over ctxs[0..count) (all in stage 1, same device; each stays
 * owned by the caller and must outlive the batch).  All batch work is
 * enqueued on hip_stream, which must not be the default stream when graphs
 * are used.  Errors: NMF_EINVAL, NMF_ENOMEM, NMF_ESTATE, NMF_EDEVICE. */
nmf_status nmf_batch_create(nmf_ctx *const *ctxs, int32_t count, void *device_workspace, size_t ws_bytes,
                            void *hip_stream, nmf_batch **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, request loops that must not call hipMalloc, harnesses that forbid
 * it): nmf_batch_create() without a caller workspace.  The batch tables live
 * in a fixed array of device memory inside the library, one copy per device
 * (batch_bytes(NMF_BATCH_STATIC_MAX), 304 KiB, held until the process
 * ends), looked up on the current device, which must be the contexts' device.
 * Nothing is allocated on the device.  The array is shared by every batch made
 * this way on that device: creating another one (or refreshing one) rewrites
 * the tables, so only the most recent such batch may be stepped or polled, and
 * calls that overlap on one device race.  Batches made with a workspace are
 * not affected.  Results are those of nmf_batch_create() on the same contexts.
 * Errors: as nmf_batch_create(); NMF_ECAPACITY when count exceeds
 * NMF_BATCH_STATIC_MAX. */
#define NMF_BATCH_STATIC_MAX 1024
nmf_status nmf_batch_create_static(nmf_ctx *const *ctxs, int32_t count, void *hip_stream, nmf_batch **out);

/* Re-reads the contexts' sizes and launch shapes (after nmf_set_launch_shape
 * or nmf_append_columns) and drops any captured graph. */
nmf_status nmf_batch_refresh(nmf_batch *b);

/* Enqueues `sweeps` stage-1 sweeps of every problem.  Problems of one rank k
 * (a K-group) share flattened launches; a batch made by nmf_batch_create()
 * runs its K-groups concurrently, each on a side stream of its own (default
 * priority) forked from and joined back to the batch's stream by events, so
 * work enqueued on the batch's stream afterwards still sees every sweep.
 * use_graph = 1 captures the sweeps into a HIP graph on first use (per sweep
 * count; the K-groups become parallel branches) and replays it.  Batches made
 * by nmf_batch_create_static() run their K-groups one after another on the
 * batch's stream. */
nmf_status nmf_batch_anls_step(nmf_batch *b, int32_t sweeps, int32_t use_graph);

/* Waits for the batch's stream, then copies every context's stage-1 state
 * out: converged[q] = 1 once context q's stop rule (Sec. IV) or its sweep
 * budget holds, sweeps[q] = its sweep count (host arrays of the batch's
 * count, in the order of nmf_batch_create's ctxs; either may be NULL).  Used
 * by request loops that retire finished problems between sweeps. */
nmf_status nmf_batch_poll(nmf_batch *b, int32_t *converged, int64_t *sweeps);

/* Waits for the batch's stream. */
nmf_status nmf_batch_sync(nmf_batch *b);

nmf_status nmf_batch_destroy(nmf_batch *b);

/* Current sizes: rows n, columns m, rank k. */
nmf_status nmf_get_shape(const nmf_ctx *ctx, int64_t *n, int64_t *m, int32_t *k);

/* Releases the context (the workspace goes back to the caller).  NULL is ok. */
nmf_status nmf_destroy(nmf_ctx *ctx);

/* Last error message of a context, or of the last failed nmf_create when ctx
 * is NULL.  Never NULL. */
const char *nmf_last_error(const nmf_ctx *ctx);

/* Name of a status code. */
const char *nmf_status_string(nmf_status status);

#ifdef __cplusplus
}
#endif

#endif /* NMF_H */
