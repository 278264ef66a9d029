"""Batched stage-1 sweeps: every problem of a batch ends bitwise where its own
standalone sweeps end, with eager launches and with HIP-graph replays."""
import numpy as np
import pytest

from paper_2101_08431_amd import synth

pytestmark = pytest.mark.gpu


def problems(count, seed0=10000):
    rng = np.random.default_rng(seed0)
    out = []
    for q in range(count):
        n = int(rng.integers(100, 900))
        m = int(rng.integers(20, 200))
        k = int(rng.integers(2, 9))
        M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-3, sigma_relative=True), seed0 + q)
        out.append((M, X0, Y0, k))
    return out


def contexts(probs, **opt):
    from paper_2101_08431_amd import NMF, default_options
    base = dict(eps_stol=-1.0, max_anls_sweeps=1 << 30, with_ipm=0)
    base.update(opt)
    return [NMF(M, k, X0, Y0, options=default_options(**base)) for (M, X0, Y0, k) in probs]


def test_batch_matches_standalone_eager_and_graph():
    import torch
    from paper_2101_08431_amd import Batch
    probs = problems(14)
    print("case batch of 14 uneven problems", flush=True)
    solo = contexts(probs)
    for c in solo:
        c.anls_step(12, report=False)
    torch.cuda.synchronize()
    ref = [c.factors() for c in solo]
    for graph in (False, True):
        ctxs = contexts(probs)
        b = Batch(ctxs)
        for _ in range(3):                       # 3 x 4 = 12 sweeps
            b.step(4, graph=graph)
            b.sync()
            torch.cuda.synchronize()             # eager work between replays
        for c, (X, Y) in zip(ctxs, ref):
            Xb, Yb = c.factors()
            assert np.array_equal(Xb, X) and np.array_equal(Yb, Y)
        b.close()


def test_batch_problems_stop_independently():
    import torch
    from paper_2101_08431_amd import Batch
    probs = problems(6, seed0=10100)
    ctxs = contexts(probs, eps_stol=1e-6, max_anls_sweeps=40)
    b = Batch(ctxs)
    b.step(50, graph=True)
    b.sync()
    torch.cuda.synchronize()
    for c in ctxs:
        st, rep = c.anls_step(0)
        assert st == 1 and rep["sweeps"] <= 40
    solo = contexts(probs, eps_stol=1e-6, max_anls_sweeps=40)
    for c, s in zip(ctxs, solo):
        s.anls_step(50)
        assert np.array_equal(c.factors()[0], s.factors()[0])


def test_batch_after_relaunch_shape_change():
    import torch
    from paper_2101_08431_amd import Batch
    probs = problems(5, seed0=10200)
    ctxs = contexts(probs)
    b = Batch(ctxs)
    b.step(3, graph=True)
    b.sync()
    for c in ctxs:
        c.set_launch_shape(2, 1)
    b.refresh()
    b.step(3, graph=True)
    b.sync()
    torch.cuda.synchronize()
    solo = contexts(probs)
    for c in solo:
        c.anls_step(3, report=False)
        c.set_launch_shape(2, 1)
        c.anls_step(3, report=False)
    torch.cuda.synchronize()
    for c, s in zip(ctxs, solo):
        assert np.array_equal(c.factors()[0], s.factors()[0])


def test_batch_poll_reports_each_problem():
    import torch
    from paper_2101_08431_amd import Batch
    probs = problems(7, seed0=10300)
    print("case batch poll, 7 problems, stop rule 1e-6, budget 30", flush=True)
    ctxs = contexts(probs, eps_stol=1e-6, max_anls_sweeps=30)
    b = Batch(ctxs)
    conv, sweeps = b.poll()
    assert not conv.any() and (sweeps == 0).all()
    b.step(5, graph=False)
    conv, sweeps = b.poll()
    for c, cv, sw in zip(ctxs, conv, sweeps):
        st, rep = c.anls_step(0)
        assert rep["sweeps"] == sw and (st == 1) == bool(cv)
    b.step(40, graph=False)
    conv, sweeps = b.poll()
    assert conv.all() and (sweeps <= 30).all()
    torch.cuda.synchronize()


def test_append_rearms_the_sweep_budget():
    # after nmf_append_columns the stop rule gets a fresh budget of
    # max_anls_sweeps sweeps, counted from the sweeps done so far
    from paper_2101_08431_amd import NMF, default_options
    M, _, _ = synth.pdf_like(300, 60, 3, 5, sigma=1e-3, sigma_relative=True)
    M = np.asarray(M)
    X0, Y0 = synth.random_init(300, 40, 3, 5, float(np.linalg.norm(M[:, :40])))
    ctx = NMF(np.asfortranarray(M[:, :40]), 3, X0, Y0, m_capacity=60,
              options=default_options(eps_stol=0.0, max_anls_sweeps=7, with_ipm=0))
    st, rep = ctx.anls_step(20)
    assert st == 1 and rep["sweeps"] == 7
    ctx.append_columns(np.asfortranarray(M[:, 40:]))
    st, rep = ctx.anls_step(3)
    assert st == 0 and rep["sweeps"] == 10
    st, rep = ctx.anls_step(20)
    assert st == 1 and rep["sweeps"] == 14
    # an explicit budget re-arms the stop rule and applies to later appends
    ctx.set_anls_budget(5)
    st, rep = ctx.anls_step(20)
    assert st == 1 and rep["sweeps"] == 19


def test_batch_many_groups_mixed_halves_with_polls():
    # seven K groups in one batch (their offset tables together exceed one
    # entry per problem), problems whose halves run as two kernels, as one
    # kernel (with one split or several) or mixed,
    # and a poll between every step: each problem still ends bitwise where
    # its standalone sweeps end
    import torch
    from paper_2101_08431_amd import Batch
    rng = np.random.default_rng(10400)
    probs, shapes = [], []
    for q in range(9):
        k = 2 + q % 7
        n, m = (1500, 300) if q % 3 == 0 else (int(rng.integers(100, 600)), int(rng.integers(20, 120)))
        M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-3, sigma_relative=True), 10400 + q)
        probs.append((M, X0, Y0, k))
        shapes.append([None, (1, 2, -1, -1), (2, 1, -1, -1), (3, 2, 1, 1), (2, 3, 0, 1)][q % 5])
    print("case batch of 9 problems over 7 K groups, two-kernel / one-kernel / mixed halves", flush=True)

    def make():
        cs = contexts(probs)
        for c, sh in zip(cs, shapes):
            if sh is not None:
                c.set_launch_shape(sh[0], sh[1])
                c.set_launch_fusion(sh[2], sh[3])
        return cs

    solo = make()
    for c in solo:
        c.anls_step(9, report=False)
    torch.cuda.synchronize()
    ctxs = make()
    b = Batch(ctxs)
    for _ in range(3):
        b.step(3, graph=False)
        conv, sweeps = b.poll()
        assert not conv.any()
    assert (sweeps == 9).all()
    torch.cuda.synchronize()
    for c, s in zip(ctxs, solo):
        assert np.array_equal(c.factors()[0], s.factors()[0])
        assert np.array_equal(c.factors()[1], s.factors()[1])
    b.close()


def test_batch_problems_match_oracle(orc):
    # uneven problems (k from 2 to 8; halves as one kernel and as split
    # kernels) swept in one batch, each against the FP64 oracle's sweeps
    import torch
    from paper_2101_08431_amd import Batch
    rng = np.random.default_rng(10300)
    probs = []
    for q in range(10):
        big = q % 3 == 0   # above 2^18 entries: split halves
        n = int(rng.integers(1200, 2400)) if big else int(rng.integers(100, 900))
        m = int(rng.integers(230, 400)) if big else int(rng.integers(20, 200))
        k = 2 + q % 7
        M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-3, sigma_relative=True), 10300 + q)
        probs.append((M, X0, Y0, k))
    print("case batch of 10 uneven problems vs oracle", flush=True)
    ctxs = contexts(probs)
    plans = [c.launch_plan() for c in ctxs]
    assert any(not p[2] for p in plans) and any(p[2] for p in plans)
    b = Batch(ctxs)
    b.step(7, graph=True)
    b.sync()
    torch.cuda.synchronize()
    for (M, X0, Y0, k), c in zip(probs, ctxs):
        X, Y = c.factors()
        ref = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=7)
        scale = max(np.abs(ref["X"]).max(), np.abs(ref["Yt"]).max())
        err = max(np.abs(X - ref["X"]).max(), np.abs(Y.T - ref["Yt"]).max()) / scale
        assert err <= 1e-8, (k, M.shape, err)
    b.close()
