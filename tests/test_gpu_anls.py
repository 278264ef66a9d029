"""Stage 1 on the GPU against the CPU oracle (same seeded inputs).

Bars: factor entries within 1e-8 of the largest entry after the same number
of sweeps; passive sets bit-exact on the small cases; bitwise-reproducible
runs; the stop rule, E(.;0) and the objective as the oracle computes them.
"""
import numpy as np
import pytest

from paper_2101_08431_amd import synth

pytestmark = pytest.mark.gpu

REL = 1e-8


def gpu_ctx(M, k, X0, Y0, m_capacity=None, **opt):
    import torch  # noqa: F401
    from paper_2101_08431_amd import NMF, default_options
    base = dict(eps_stol=-1.0, max_anls_sweeps=1 << 30)
    base.update(opt)
    return NMF(M, k, X0, Y0, m_capacity=m_capacity, options=default_options(**base))


def rel_err(X, Y, Xr, Ytr):
    scale = max(np.abs(Xr).max(), np.abs(Ytr).max(), 1e-300)
    return max(np.abs(X - Xr).max(), np.abs(Y.T - Ytr).max()) / scale


def spec(n, m, k, sigma=1e-3, rel=False):
    return dict(kind="pdf", n=n, m=m, k=k, sigma=sigma, sigma_relative=rel)


@pytest.mark.parametrize("sweeps", [1, 5, 20])
def test_sweeps_match_oracle_200x50x3(orc, sweeps):
    M, X0, Y0 = synth.make("pdf_200x50_k3", 0)
    print(f"case pdf_200x50_k3 seed 0 sweeps {sweeps}", flush=True)
    ctx = gpu_ctx(M, 3, X0, Y0)
    ctx.anls_step(sweeps)
    X, Y = ctx.factors()
    xm, ym = ctx.masks()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=sweeps)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL
    assert np.array_equal(xm, ref["xmask"]) and np.array_equal(ym, ref["ymask"])
    assert np.all(X >= 0) and np.all(Y >= 0)


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (5, 3, 2), (63, 17, 1), (65, 64, 2), (130, 37, 4),
                                   (257, 129, 7), (300, 90, 10), (129, 70, 13), (200, 40, 16)])
def test_ragged_shapes_match_oracle(orc, n, m, k):
    print(f"case ragged n={n} m={m} k={k}", flush=True)
    M, X0, Y0 = synth.make(spec(n, m, k, 1e-2), 3)
    ctx = gpu_ctx(M, k, X0, Y0)
    ctx.anls_step(4)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=4)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL


@pytest.mark.parametrize("shape", [(1, 1, -1, -1), (1, 3, -1, -1), (8, 1, -1, -1), (8, 3, -1, -1),
                                   (64, 64, -1, -1), (8, 3, 1, 1), (3, 8, 1, 0), (64, 64, 1, 1), (1, 1, 0, 0),
                                   (2, 5, 0, 1)])
def test_launch_shapes_match_oracle(orc, shape):
    # each half as one kernel (the tile's last split solves) or as a split
    # stream + NNLS kernel, on a ragged size with several tiles; every launch
    # plan reaches the oracle's iterates
    n, m, k = 1100, 230, 5
    print(f"case launch plan {shape} n={n} m={m} k={k}", flush=True)
    M, X0, Y0 = synth.make(spec(n, m, k, 1e-3, True), 12)
    ctx = gpu_ctx(M, k, X0, Y0, x_splits=shape[0], y_splits=shape[1])
    ctx.set_launch_fusion(shape[2], shape[3])
    plan = ctx.launch_plan()
    assert plan[2] == (shape[0] == 1 if shape[2] < 0 else bool(shape[2]))
    assert plan[3] == (shape[1] == 1 if shape[3] < 0 else bool(shape[3]))
    ctx.anls_step(6)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=6)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL
    # switching the plan in the middle of a run keeps the iterates
    ctx.set_launch_shape(shape[1], shape[0])
    ctx.set_launch_fusion(shape[3], shape[2])
    ctx.anls_step(3)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=9)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL


def test_full_size_3000x500x5(orc):
    print("case pdf_3000x500_k5 seed 0 sweeps 10", flush=True)
    M, X0, Y0 = synth.make("pdf_3000x500_k5", 0)
    ctx = gpu_ctx(M, 5, X0, Y0)
    ctx.anls_step(10)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=10)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL
    xm, ym = ctx.masks()
    # passive sets agree except where an entry sits within rounding of zero
    close = np.abs(ref["X"]).min(axis=1) > 1e-9 * np.abs(ref["X"]).max()
    assert np.array_equal(xm[close], ref["xmask"][close])


def test_full_size_10000x2000x10(orc):
    print("case pdf_10000x2000_k10 seed 0 sweeps 3", flush=True)
    M, X0, Y0 = synth.make("pdf_10000x2000_k10", 0)
    ctx = gpu_ctx(M, 10, X0, Y0)
    ctx.anls_step(3)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=3)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL


def test_bitwise_reproducible():
    M, X0, Y0 = synth.make("pdf_3000x500_k5", 1)
    outs = []
    for _ in range(2):
        ctx = gpu_ctx(M, 5, X0, Y0)
        ctx.anls_step(7)
        outs.append(ctx.factors())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_stop_rule_and_report_match_oracle(orc):
    M, X0, Y0 = synth.make("pdf_200x50_k3", 1)
    ctx = gpu_ctx(M, 3, X0, Y0, eps_stol=1e-6, max_anls_sweeps=5000)
    st, rep = ctx.anls_step(5000)
    ref = orc.anls(M, X0, Y0.T.copy(), eps_stol=1e-6, max_sweeps=5000)
    assert st == 1 and ref["met"]
    assert abs(rep["sweeps"] - ref["sweeps"]) <= 1
    # further sweeps are no-ops once the rule holds
    X1, Y1 = ctx.factors()
    ctx.anls_step(10)
    X2, Y2 = ctx.factors()
    assert np.array_equal(X1, X2) and np.array_equal(Y1, Y2)
    r = ctx.report()
    f = orc.objective(M, X1, Y1.T.copy())
    E = orc.kkt_error_anls(M, X1, Y1.T.copy())
    assert r["f"] == pytest.approx(f, rel=1e-10)
    assert r["E0"] == pytest.approx(E, rel=1e-6, abs=1e-14)


def test_append_columns_warm_start(orc):
    n, k, m0, add, horizon = 400, 4, 64, 16, 96
    M, _, _ = synth.pdf_like(n, horizon, k, 5, sigma=1e-3, sigma_relative=True)
    M = np.asarray(M)
    X0, Y0 = synth.random_init(n, m0, k, 5, float(np.linalg.norm(M[:, :m0])))
    ctx = gpu_ctx(np.asfortranarray(M[:, :m0]), k, X0, Y0, m_capacity=horizon)
    ctx.anls_step(30)
    X, Y = ctx.factors()
    ctx.append_columns(np.asfortranarray(M[:, m0:m0 + add]))
    assert ctx.m == m0 + add
    X2, Y2 = ctx.factors()
    assert np.array_equal(X2, X)
    # the appended columns are the NNLS solutions given X (unique, so any
    # warm start gives them)
    Yt_ref, _, _ = orc.half_y(np.asfortranarray(M[:, :m0 + add]), X, np.zeros((m0 + add, k)))
    assert np.abs(Y2.T - Yt_ref).max() <= REL * np.abs(Yt_ref).max()
    # sweeps continue on the grown problem and match the oracle from there
    ctx.anls_step(5)
    X3, Y3 = ctx.factors()
    ref = orc.anls(np.asfortranarray(M[:, :m0 + add]), X2, Y2.T.copy(), exact_sweeps=5)
    assert rel_err(X3, Y3, ref["X"], ref["Yt"]) <= REL
    with pytest.raises(Exception, match="ECAPACITY"):
        ctx.append_columns(np.asfortranarray(M[:, :add + 1]))


def test_device_resident_inputs(orc):
    import torch
    M, X0, Y0 = synth.make("pdf_200x50_k3", 2)
    Md = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
    ctx = gpu_ctx(Md, 3, torch.from_numpy(X0).cuda(), torch.from_numpy(Y0).cuda())
    ctx.anls_step(6)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=6)
    assert rel_err(X, Y, ref["X"], ref["Yt"]) <= REL


def test_invalid_inputs_rejected():
    from paper_2101_08431_amd import NMFError
    M, X0, Y0 = synth.make("pdf_200x50_k3", 0)
    bad = M.copy(order="F")
    bad[3, 4] = np.nan
    with pytest.raises(NMFError, match="EINVAL"):
        gpu_ctx(bad, 3, X0, Y0)
    Xn = X0.copy()
    Xn[0, 0] = -1.0
    with pytest.raises(NMFError, match="EINVAL"):
        gpu_ctx(M, 3, Xn, Y0)


def test_seeded_start_without_x0():
    from paper_2101_08431_amd import NMF, default_options
    M, _, _ = synth.make("pdf_200x50_k3", 0)
    ctx = NMF(M, 3, options=default_options(seed=5))
    X, Y = ctx.factors()
    assert np.all(X >= 0) and np.all(Y >= 0)
    assert np.linalg.norm(X @ Y) == pytest.approx(np.linalg.norm(M), rel=1e-12)


@pytest.mark.parametrize("prec,tol", [(1, 2e-5), (2, 5e-4)])
def test_reduced_precision_gram_sweeps(orc, prec, tol):
    # FP32 or BF16 hi+lo copies of M in the two streaming products, FP32
    # accumulation; the NNLS stays FP64.  The error against the FP64 oracle
    # after a few sweeps is bounded by the input rounding (2^-24, resp. about
    # 2^-16 relative per element) amplified by the conditioning of the sweep.
    M, X0, Y0 = synth.make("pdf_3000x500_k5", 0)
    print(f"case precision {prec} pdf_3000x500_k5 sweeps 5", flush=True)
    ctx = gpu_ctx(M, 5, X0, Y0, gram_precision=prec)
    ctx.anls_step(5)
    X, Y = ctx.factors()
    ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=5)
    err = rel_err(X, Y, ref["X"], ref["Yt"])
    print(f"precision {prec}: max factor error vs FP64 oracle {err:.3e}", flush=True)
    assert err <= tol
    assert err > 0.0      # the reduced path really ran


def test_reduced_precision_solve_reaches_fp64_kkt(orc):
    from paper_2101_08431_amd import NMF, default_options
    M, X0, Y0 = synth.make("pdf_200x50_k3", 1)
    out = {}
    for prec in (0, 1, 2):
        ctx = NMF(M, 3, X0, Y0, options=default_options(eps_tol=1e-10, gram_precision=prec))
        st, rep = ctx.solve()
        assert st == 1 and rep["E0"] <= 1e-10
        X, Y = ctx.factors()
        out[prec] = orc.objective(M, X, Y.T.copy())
    assert abs(out[1] - out[0]) <= 1e-10 * out[0]
    assert abs(out[2] - out[0]) <= 1e-10 * out[0]
