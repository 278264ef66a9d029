"""Mixed-precision interior point (nmf_set_ipm_precision) against the CPU
oracle.

With mixed = 1 the exact-Hessian Schur complement of eq. (27) is formed on
FP32 matrix cores and every direction solved with its factor is refined
against the FP64 operator.  Alg. 3 is unchanged, so a converged solve lands on
the oracle's end point: objective within 1e-10 and E(.;0) re-derived from the
GPU's own iterate and duals; normalised factors within 1e-8 where the
exact-Hessian decisions match the oracle's (200x50x3), within 5e-6 at
3000x500x5 where they do not (measured 8.6e-7); the mixed and FP64 solves
from one point agree (their iteration and exact-step counts are printed)."""
import os

import numpy as np
import pytest

from paper_2101_08431_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "solve_pdf_3000x500_k5_seed0.npz")
# normalised-factor bar at 3000x500x5, where the mixed path's exact-Hessian
# decisions differ from the oracle's (see the test)
MIXED_FACTOR_BAR = 5e-6


def rel(A, B):
    return float(np.abs(A - B).max() / max(np.abs(B).max(), 1e-300))


def start_point(orc, name, seed):
    M, X0, Y0 = synth.make(name, seed)
    r = orc.anls(M, X0, Y0.T.copy(), eps_stol=1e-6, max_sweeps=5000)
    return np.asarray(M), r["X"], r["Yt"]


def gpu_ctx(M, X, Yt, mixed, **opt):
    from paper_2101_08431_amd import NMF, default_options
    base = dict(eps_stol=-1.0, max_anls_sweeps=1 << 30)
    base.update(opt)
    ctx = NMF(np.asfortranarray(M), X.shape[1], np.ascontiguousarray(X), np.ascontiguousarray(Yt.T),
              options=default_options(**base))
    ctx.set_ipm_precision(mixed, 2)
    return ctx


@pytest.mark.parametrize("seed", [0, 1, 4])
def test_mixed_full_solve_200x50x3_matches_oracle(orc, seed):
    M, X, Yt = start_point(orc, "pdf_200x50_k3", seed)
    print(f"case mixed full solve pdf_200x50_k3 seed {seed}", flush=True)
    ctx = gpu_ctx(M, X, Yt, 1, eps_tol=1e-10)
    st, rep = ctx.ipm_step(1000)
    assert st == 1, rep
    assert rep["exact_steps"] > 0
    Xg, Yg = ctx.factors()
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-10)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, orc.IPMOptions(eps_tol=1e-10))
    assert res.converged
    fg = orc.objective(M, Xg, Yg.T.copy())
    fo = orc.objective(M, res.X, res.Yt)
    Xn, Yn = orc.normalise(Xg, Yg.T)
    Xon, Yon = orc.normalise(res.X, res.Yt)
    print(f"mixed end-point agreement: f {abs(fg - fo) / fo:.2e}, normalised X {rel(Xn, Xon):.2e}, "
          f"Y {rel(Yn, Yon):.2e}; exact steps {rep['exact_steps']}", flush=True)
    assert abs(fg - fo) <= 1e-10 * fo + 1e-16 * 0.5 * np.sum(M * M)
    assert rel(Xn, Xon) <= 1e-8 and rel(Yn, Yon) <= 1e-8
    Rg, Sg = ctx.duals()
    gx, gy, _ = orc.gradients(M, Xg, Yg.T)
    assert orc.kkt_error(Xg, Yg.T, Rg, Sg.T, 0.0, gx, gy) <= 2e-10
    ctx.close()


def test_mixed_solve_3000x500x5_matches_oracle_golden(orc):
    g = np.load(GOLDEN)
    M, _, _ = synth.make("pdf_3000x500_k5", 0)
    M = np.asarray(M)
    print("case mixed golden solve pdf_3000x500_k5 seed 0 to 1e-10", flush=True)
    ctx = gpu_ctx(M, g["X1"], g["Yt1"], 1, eps_tol=1e-10, max_ipm_iters=3000)
    st, rep = ctx.ipm_step(3000)
    print({k: rep[k] for k in ("E0", "f", "ipm_iters", "ipm_outer", "exact_steps", "fallbacks")}, flush=True)
    assert st == 1 and rep["E0"] <= 1e-10, rep
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    gx, gy, _ = orc.gradients(M, Xg, Yg.T)
    assert orc.kkt_error(Xg, Yg.T, Rg, Sg.T, 0.0, gx, gy) <= 2e-10
    fg = orc.objective(M, Xg, Yg.T.copy())
    f_err = abs(fg - float(g["f"])) / float(g["f"])
    Xn, Yn = orc.normalise(Xg, Yg.T)
    Xon, Yon = orc.normalise(g["X"], g["Yt"])
    print(f"mixed golden agreement: f {f_err:.2e}, normalised X {rel(Xn, Xon):.2e}, Y {rel(Yn, Yon):.2e}",
          flush=True)
    assert f_err <= 1e-10
    # The FP32-formed exact-Hessian matrix stops factoring near the end more
    # often than the FP64 one (each failure is the fallback to the
    # Gauss-Newton matrix of Alg. 3), so this path differs from the oracle's
    # and stops at another point with E(.;0) <= 1e-10.  Points that meet that
    # bound lie within about E / lambda_min of the minimiser; measured: 8.6e-7
    # on the normalised factors, with the objective equal to the last digit.
    assert rel(Xn, Xon) <= MIXED_FACTOR_BAR and rel(Yn, Yon) <= MIXED_FACTOR_BAR
    ctx.close()


def test_mixed_and_fp64_solves_agree(orc):
    # the same solve in both precisions from the same point: the iteration
    # and exact-step counts are printed, the end points must agree
    M, X, Yt = start_point(orc, "pdf_200x50_k3", 1)
    print("case mixed vs fp64 solve pdf_200x50_k3 seed 1", flush=True)
    out = []
    for mixed in (0, 1):
        ctx = gpu_ctx(M, X, Yt, mixed, eps_tol=1e-10)
        st, rep = ctx.ipm_step(1000)
        assert st == 1, rep
        Xg, Yg = ctx.factors()
        out.append((orc.objective(M, Xg, Yg.T.copy()), orc.normalise(Xg, Yg.T), rep["ipm_iters"], rep["exact_steps"]))
        ctx.close()
    (f0, (X0n, Y0n), it0, ex0), (f1, (X1n, Y1n), it1, ex1) = out
    print(f"fp64: {it0} iterations, {ex0} exact steps; mixed: {it1} iterations, {ex1} exact steps; "
          f"f {abs(f1 - f0) / f0:.2e}, X {rel(X1n, X0n):.2e}, Y {rel(Y1n, Y0n):.2e}", flush=True)
    assert abs(f1 - f0) <= 1e-10 * f0
    assert rel(X1n, X0n) <= 1e-8 and rel(Y1n, Y0n) <= 1e-8
