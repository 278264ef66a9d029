"""Stage 2 (transition and interior-point iterations) on the GPU against the
CPU oracle, from the same starting point.

The starting point is the oracle's own stage-1 end point (inputs flow from the
oracle to the GPU, never back).  The transition is deterministic and is
compared entry by entry; a few IPM iterations are compared as trajectories
(the Armijo decisions agree away from rounding ties); converged end points are
compared after removing the scaling freedom, and certified independently by
the KKT conditions eq. (3).
"""
import os

import numpy as np
import pytest

from paper_2101_08431_amd import synth

pytestmark = pytest.mark.gpu

# Agreement of normalised end points with the oracle's (the spec bar on
# factor entries); measured: about 1e-11 at 3000x500x5, 1e-15 at 200x50x3.
GOLDEN_FACTOR_BAR = 1e-8


def start_point(orc, name, seed, sweeps=None, eps_stol=1e-6):
    M, X0, Y0 = synth.make(name, seed)
    if sweeps is None:
        r = orc.anls(M, X0, Y0.T.copy(), eps_stol=eps_stol, max_sweeps=5000)
    else:
        r = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=sweeps)
    return np.asarray(M), r["X"], r["Yt"]


def gpu_ctx(M, X, Yt, **opt):
    from paper_2101_08431_amd import NMF, default_options
    base = dict(eps_stol=-1.0, max_anls_sweeps=1 << 30)
    base.update(opt)
    return NMF(np.asfortranarray(M), X.shape[1], np.ascontiguousarray(X), np.ascontiguousarray(Yt.T),
               options=default_options(**base))


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_transition_matches_oracle(orc):
    M, X, Yt = start_point(orc, "pdf_200x50_k3", 0)
    print("case transition pdf_200x50_k3 seed 0", flush=True)
    ctx = gpu_ctx(M, X, Yt, eps_tol=1e-10)
    st, rep = ctx.ipm_step(0)
    Xo, Yo, ro, so, muo, rhoo = orc.transition(M, X, Yt, 1e-10)
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    assert rel(Xg, Xo) <= 1e-14 and rel(Yg.T, Yo) <= 1e-14
    assert rel(Rg, ro) <= 1e-10 and rel(Sg.T, so) <= 1e-10
    assert rep["mu"] == pytest.approx(muo, rel=1e-10)
    gx, gy, _ = orc.gradients(M, Xo, Yo)
    assert rep["E0"] == pytest.approx(orc.kkt_error(Xo, Yo, ro, so, 0.0, gx, gy), rel=1e-8)
    assert rep["Emu"] == pytest.approx(orc.kkt_error(Xo, Yo, ro, so, muo, gx, gy), rel=1e-8)


@pytest.mark.parametrize("name,seed,iters", [("pdf_200x50_k3", 0, 1), ("pdf_200x50_k3", 0, 3),
                                             ("pdf_200x50_k3", 1, 6)])
def test_first_iterations_match_oracle(orc, name, seed, iters):
    M, X, Yt = start_point(orc, name, seed)
    print(f"case ipm iterations {name} seed {seed} iters {iters}", flush=True)
    ctx = gpu_ctx(M, X, Yt, eps_tol=1e-10)
    ctx.ipm_step(iters)
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    opts = orc.IPMOptions(eps_tol=1e-10, max_inner=iters)
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-10)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, opts)
    assert res.inner == iters
    print(f"trajectory agreement: X {rel(Xg, res.X):.2e} Y {rel(Yg.T, res.Yt):.2e} "
          f"R {rel(Rg, res.r):.2e} S {rel(Sg.T, res.s):.2e}", flush=True)
    assert rel(Xg, res.X) <= 1e-8 and rel(Yg.T, res.Yt) <= 1e-8
    assert rel(Rg, res.r) <= 1e-8 and rel(Sg.T, res.s) <= 1e-8


@pytest.mark.parametrize("k", [6, 7, 8, 9, 12, 16])
def test_first_iteration_across_ranks_matches_oracle(orc, k):
    # the Gauss-Newton formation splits the K(K+1)/2 products (a, b) into a
    # rank-dependent number of chunks, prefetch depth and staging height;
    # these ranks cover every such plan (m = 70: a ragged last tile)
    spec = dict(kind="pdf", n=150, m=70, k=k, sigma=1e-3, sigma_relative=True)
    M, X, Yt = start_point(orc, spec, 3, sweeps=40)
    print(f"case ipm first iteration pdf 150x70 k={k}", flush=True)
    ctx = gpu_ctx(M, X, Yt, eps_tol=1e-10)
    ctx.ipm_step(1)
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    ctx.close()
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-10)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, orc.IPMOptions(eps_tol=1e-10, max_inner=1))
    assert res.inner == 1
    print(f"k={k} agreement: X {rel(Xg, res.X):.2e} Y {rel(Yg.T, res.Yt):.2e} "
          f"R {rel(Rg, res.r):.2e} S {rel(Sg.T, res.s):.2e}", flush=True)
    assert rel(Xg, res.X) <= 1e-8 and rel(Yg.T, res.Yt) <= 1e-8
    assert rel(Rg, res.r) <= 1e-8 and rel(Sg.T, res.s) <= 1e-8


def test_exact_hessian_slabs_and_split_rank_update_match_oracle(orc):
    # n k = 70000 rows of V: two slabs of at most 65535 rows; mk = 300: six
    # 128 x 128 tiles, so the rank update splits the rows of each slab over
    # several blocks per tile.  sigma_c = 1 turns the exact Hessian (eq. (27))
    # on at the first mu update, so iterations 4-6 take exact steps.
    spec = dict(kind="pdf", n=14000, m=60, k=5, sigma=1e-3, sigma_relative=True)
    M, X, Yt = start_point(orc, spec, 2, sweeps=30)
    print("case exact-Hessian slabs + split rank update 14000x60x5", flush=True)
    ctx = gpu_ctx(M, X, Yt, eps_tol=1e-10, sigma_c=1.0)
    _, rep = ctx.ipm_step(6)
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    ctx.close()
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-10)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, orc.IPMOptions(eps_tol=1e-10, max_inner=6, sigma_c=1.0))
    assert res.inner == 6 and res.exact_steps == 3
    print(f"exact steps gpu {rep['exact_steps']} oracle {res.exact_steps}; agreement: X {rel(Xg, res.X):.2e} "
          f"Y {rel(Yg.T, res.Yt):.2e} R {rel(Rg, res.r):.2e} S {rel(Sg.T, res.s):.2e}", flush=True)
    assert rep["exact_steps"] == res.exact_steps
    assert rel(Xg, res.X) <= 1e-8 and rel(Yg.T, res.Yt) <= 1e-8
    assert rel(Rg, res.r) <= 1e-8 and rel(Sg.T, res.s) <= 1e-8


@pytest.mark.parametrize("seed", [0, 1, 4])
def test_full_solve_200x50x3_matches_oracle(orc, seed):
    M, X, Yt = start_point(orc, "pdf_200x50_k3", seed)
    print(f"case full solve pdf_200x50_k3 seed {seed}", flush=True)
    ctx = gpu_ctx(M, X, Yt, eps_tol=1e-10)
    st, rep = ctx.ipm_step(1000)
    assert st == 1, rep
    Xg, Yg = ctx.factors()
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-10)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, orc.IPMOptions(eps_tol=1e-10))
    assert res.converged
    fg = orc.objective(M, Xg, Yg.T.copy())
    fo = orc.objective(M, res.X, res.Yt)
    assert abs(fg - fo) <= 1e-10 * fo + 1e-16 * 0.5 * np.sum(M * M)
    Xn, Yn = orc.normalise(Xg, Yg.T)
    Xon, Yon = orc.normalise(res.X, res.Yt)
    print(f"end-point agreement: f {abs(fg - fo) / fo:.2e}, normalised X {rel(Xn, Xon):.2e}, "
          f"Y {rel(Yn, Yon):.2e}", flush=True)
    assert rel(Xn, Xon) <= 1e-8 and rel(Yn, Yon) <= 1e-8
    # independent certificate: E(.;0) from the GPU's own iterate and duals
    Rg, Sg = ctx.duals()
    gx, gy, _ = orc.gradients(M, Xg, Yg.T)
    assert orc.kkt_error(Xg, Yg.T, Rg, Sg.T, 0.0, gx, gy) <= 2e-10
    assert rep["E0"] <= 1e-10


def test_nmf_solve_two_stages_200x50x3(orc):
    M, X0, Y0 = synth.make("pdf_200x50_k3", 2)
    from paper_2101_08431_amd import NMF, default_options
    ctx = NMF(np.asarray(M), 3, X0, Y0, options=default_options(eps_tol=1e-10))
    st, rep = ctx.solve()
    assert st == 1 and rep["stage"] == 2 and rep["E0"] <= 1e-10
    ref = orc.solve(np.asarray(M), X0, Y0.T.copy(), orc.IPMOptions(eps_tol=1e-10))
    assert ref["converged"]
    Xg, Yg = ctx.factors()
    fg = orc.objective(M, Xg, Yg.T.copy())
    assert abs(fg - ref["f"]) <= 1e-10 * ref["f"]
    assert abs(rep["sweeps"] - ref["stage1"]["sweeps"]) <= 1


def test_separable_recovery_gpu(orc):
    n, m, k = 40, 20, 3
    M, xs, ys = synth.separable(n, m, k, 3)
    X0, Y0 = synth.perturbed_init(xs, ys, 3, 0.1)
    from paper_2101_08431_amd import NMF, default_options
    ctx = NMF(np.asarray(M), k, X0, Y0, options=default_options(eps_tol=1e-10))
    st, rep = ctx.solve()
    assert st == 1
    Xg, Yg = ctx.factors()
    assert orc.objective(M, Xg, Yg.T.copy()) <= 1e-14 * 0.5 * np.sum(np.asarray(M) ** 2)
    Xn, Ytn = orc.normalise(Xg, Yg.T)
    Xt, Ytt = orc.normalise(xs, ys.T)
    perm = [int(np.argmax(np.abs(Xn.T @ Xt[:, a]))) for a in range(k)]
    assert sorted(perm) == list(range(k))
    np.testing.assert_allclose(Xn[:, perm], Xt, atol=1e-6)


def test_first_iteration_3000x500x5_matches_oracle(orc):
    # full-size parity: the same stage-1 end point, then the transition and one
    # interior-point iteration on both sides
    M, X, Yt = start_point(orc, "pdf_3000x500_k5", 1, sweeps=300)
    print("case ipm 1 iteration pdf_3000x500_k5 seed 1", flush=True)
    ctx = gpu_ctx(M, X, Yt, eps_tol=1e-8)
    ctx.ipm_step(1)
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-8)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, orc.IPMOptions(eps_tol=1e-8, max_inner=1))
    print(f"trajectory agreement: X {rel(Xg, res.X):.2e} Y {rel(Yg.T, res.Yt):.2e} "
          f"R {rel(Rg, res.r):.2e} S {rel(Sg.T, res.s):.2e}", flush=True)
    assert rel(Xg, res.X) <= 1e-8 and rel(Yg.T, res.Yt) <= 1e-8
    assert rel(Rg, res.r) <= 1e-8 and rel(Sg.T, res.s) <= 1e-8


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "solve_pdf_3000x500_k5_seed0.npz")


def test_solve_3000x500x5_matches_oracle_golden(orc):
    # Alg. 3 at full size from the oracle's stage-1 end point (stored by
    # tests/golden/make_solve_golden.py, which calls only the oracle): the GPU
    # must converge to E(.;0) <= 1e-10 within a cap well above the oracle's
    # 458 iterations, certify it independently (eq. (10) from its own iterate
    # and duals), and land on the oracle's end point
    g = np.load(GOLDEN)
    M, _, _ = synth.make("pdf_3000x500_k5", 0)
    M = np.asarray(M)
    print("case golden solve pdf_3000x500_k5 seed 0 to 1e-10", flush=True)
    ctx = gpu_ctx(M, g["X1"], g["Yt1"], eps_tol=1e-10, max_ipm_iters=3000)
    st, rep = ctx.ipm_step(3000)
    print({k: rep[k] for k in ("E0", "f", "ipm_iters", "ipm_outer", "exact_steps", "fallbacks")}, flush=True)
    assert st == 1 and rep["E0"] <= 1e-10, rep
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    gx, gy, _ = orc.gradients(M, Xg, Yg.T)
    assert orc.kkt_error(Xg, Yg.T, Rg, Sg.T, 0.0, gx, gy) <= 2e-10
    assert np.all(Xg > 0) and np.all(Yg > 0)
    fg = orc.objective(M, Xg, Yg.T.copy())
    f_err = abs(fg - float(g["f"])) / float(g["f"])
    Xn, Yn = orc.normalise(Xg, Yg.T)
    Xon, Yon = orc.normalise(g["X"], g["Yt"])
    x_err, y_err = rel(Xn, Xon), rel(Yn, Yon)
    print(f"golden agreement: f {f_err:.2e}, normalised X {x_err:.2e}, Y {y_err:.2e}", flush=True)
    assert f_err <= 1e-10
    assert x_err <= GOLDEN_FACTOR_BAR and y_err <= GOLDEN_FACTOR_BAR


def test_first_iteration_10000x2000x10_matches_oracle_golden(orc):
    # the largest stage-2 case (Schur order 20000, S of 3.2 GB): the oracle's
    # 20-sweep stage-1 point, the transition and one interior-point iteration,
    # against the oracle's iteration stored by
    # tests/golden/make_ipm_first_golden.py (oracle only)
    g = np.load(os.path.join(os.path.dirname(GOLDEN), "ipm1_pdf_10000x2000_k10_seed0.npz"))
    M, X0, Y0 = synth.make("pdf_10000x2000_k10", 0)
    M = np.asarray(M)
    r1 = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=int(g["sweeps"]))
    print("case ipm 1 iteration pdf_10000x2000_k10 seed 0 (golden)", flush=True)
    ctx = gpu_ctx(M, r1["X"], r1["Yt"], eps_tol=float(g["eps_tol"]))
    ctx.ipm_step(1)
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    print(f"trajectory agreement: X {rel(Xg, g['X']):.2e} Y {rel(Yg.T, g['Yt']):.2e} "
          f"R {rel(Rg, g['r']):.2e} S {rel(Sg.T, g['s']):.2e}", flush=True)
    assert rel(Xg, g["X"]) <= 1e-8 and rel(Yg.T, g["Yt"]) <= 1e-8
    assert rel(Rg, g["r"]) <= 1e-8 and rel(Sg.T, g["s"]) <= 1e-8


def test_nmf_solve_3000x500x5_converges(orc):
    # the whole two-stage solve from the seeded start must converge (cap far
    # above the measured iteration counts) and certify E(.;0) <= 1e-8
    M, X0, Y0 = synth.make("pdf_3000x500_k5", 1)
    print("case nmf_solve pdf_3000x500_k5 seed 1 to 1e-8", flush=True)
    from paper_2101_08431_amd import NMF, default_options
    ctx = NMF(np.asarray(M), 5, X0, Y0, options=default_options(eps_tol=1e-8, max_ipm_iters=5000))
    st, rep = ctx.solve()
    print({k: rep[k] for k in ("E0", "f", "sweeps", "ipm_iters", "exact_steps")}, flush=True)
    assert st == 1 and rep["E0"] <= 1e-8
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    gx, gy, _ = orc.gradients(np.asarray(M), Xg, Yg.T)
    E = orc.kkt_error(Xg, Yg.T, Rg, Sg.T, 0.0, gx, gy)
    assert E == pytest.approx(rep["E0"], rel=1e-5, abs=1e-12)
    assert E <= 1.01e-8
    assert np.all(Xg > 0) and np.all(Yg > 0)


def test_append_after_stage2_returns_to_stage1(orc):
    n, k, m0, add = 300, 3, 40, 16
    M, _, _ = synth.pdf_like(n, m0 + add, k, 9, sigma=1e-3, sigma_relative=True)
    M = np.asarray(M)
    X0, Y0 = synth.random_init(n, m0, k, 9, float(np.linalg.norm(M[:, :m0])))
    from paper_2101_08431_amd import NMF, default_options
    ctx = NMF(np.asfortranarray(M[:, :m0]), k, X0, Y0, m_capacity=m0 + add,
              options=default_options(eps_tol=1e-9))
    st, rep = ctx.solve()
    assert st == 1
    ctx.append_columns(np.asfortranarray(M[:, m0:]))
    assert ctx.m == m0 + add
    st, rep = ctx.solve()
    assert st == 1 and rep["E0"] <= 1e-9
    Xg, Yg = ctx.factors()
    Rg, Sg = ctx.duals()
    gx, gy, _ = orc.gradients(M, Xg, Yg.T)
    assert orc.kkt_error(Xg, Yg.T, Rg, Sg.T, 0.0, gx, gy) <= 2e-9


def test_breakdown_leaves_a_finite_iterate():
    # seed 5 of 3000x500x5 ends in a numerical breakdown (mu falls to the
    # denormal range while E(.;0) is still 7e-6 and the Gauss-Newton matrix
    # stops factoring).  The library must report it (NMF_ESINGULAR) and keep
    # the last valid iterate: no NaN or infinity may reach X, Y or the report.
    from paper_2101_08431_amd import NMF, default_options
    from paper_2101_08431_amd._lib import NMFError
    M, X0, Y0 = synth.make("pdf_3000x500_k5", 5)
    print("case breakdown pdf_3000x500_k5 seed 5", flush=True)
    ctx = NMF(np.asarray(M), 5, X0, Y0, options=default_options(eps_tol=1e-8, max_ipm_iters=5000))
    try:
        st, rep = ctx.solve()
    except NMFError as e:
        st, rep = e.status, ctx.report()
    print(f"status {st}, E0 {rep['E0']:.3e}, iterations {rep['ipm_iters']}", flush=True)
    assert st in (1, -5), st
    X, Y = ctx.factors()
    ctx.close()
    assert np.isfinite(X).all() and np.isfinite(Y).all()
    assert (X >= 0).all() and (Y >= 0).all()
    assert np.isfinite(rep["E0"]) and np.isfinite(rep["f"])
