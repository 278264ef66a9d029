"""Pins for the oracle's ANLS stage (Sec. II, Alg. 1, stop rule of Sec. IV)."""
import numpy as np
import pytest
from scipy.optimize import nnls as scipy_nnls

from paper_2101_08431_amd import synth


def small_problem(seed=0, n=30, m=12, k=3):
    M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-2), seed)
    return np.asarray(M), X0, Y0.T.copy()


def test_objective_matches_numpy(orc):
    M, X, Yt = small_problem(1)
    f = orc.objective(M, X, Yt)
    assert f == pytest.approx(0.5 * np.sum((X @ Yt.T - M) ** 2), rel=1e-13)


def test_half_steps_match_scipy_rowwise(orc):
    # Each half-step of Alg. 1 is a set of independent eq. (2) problems:
    # rows of X with C = Y^T, d = row of M; columns of Y with C = X, d = column.
    M, X, Yt = small_problem(2)
    Xn, xm, bad = orc.half_x(M, X, Yt)
    assert bad == 0
    for i in range(M.shape[0]):
        xs, _ = scipy_nnls(Yt, M[i, :])
        np.testing.assert_allclose(Xn[i], xs, rtol=1e-8, atol=1e-12 * max(1, np.abs(xs).max()))
        assert xm[i] == sum(1 << a for a in range(X.shape[1]) if Xn[i, a] > 0)
    Yn, ym, bad = orc.half_y(M, Xn, Yt)
    assert bad == 0
    for j in range(M.shape[1]):
        ys, _ = scipy_nnls(Xn, M[:, j])
        np.testing.assert_allclose(Yn[j], ys, rtol=1e-8, atol=1e-12 * max(1, np.abs(ys).max()))


def test_half_step_exact_on_integer_data(orc):
    # With small-integer data and an interior solution every Gram entry is an
    # exact integer and the single Cholesky solve reproduces the closed form.
    Yt = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])     # Y = [[1,0,1],[0,1,1]]
    Xtrue = np.array([[1.0, 2.0], [3.0, 1.0]])
    M = Xtrue @ Yt.T
    Xn, xm, _ = orc.half_x(M, np.ones((2, 2)), Yt)
    np.testing.assert_allclose(Xn, Xtrue, rtol=1e-15)
    assert list(xm) == [3, 3]


def test_objective_monotone_over_half_steps(orc):
    # Each half-step is an exact block minimisation, so f never increases.
    M, X, Yt = small_problem(3, n=60, m=25, k=4)
    f_prev = orc.objective(M, X, Yt)
    for _ in range(30):
        X, _, _ = orc.half_x(M, X, Yt)
        f1 = orc.objective(M, X, Yt)
        Yt, _, _ = orc.half_y(M, X, Yt)
        f2 = orc.objective(M, X, Yt)
        assert f1 <= f_prev * (1 + 1e-13) + 1e-300
        assert f2 <= f1 * (1 + 1e-13) + 1e-300
        f_prev = f2


def test_half_step_satisfies_subproblem_kkt(orc):
    # After the X-half, grad_X f = X (Y Y^T) - M Y^T is zero on X > 0 and
    # non-negative on X = 0 (KKT of eq. (2) for every row).
    M, X, Yt = small_problem(4, n=80, m=20, k=4)
    X, _, _ = orc.half_x(M, X, Yt)
    g = X @ (Yt.T @ Yt) - M @ Yt
    scale = np.abs(M @ Yt).max()
    assert np.all(g[X > 0] <= 1e-11 * scale) and np.all(g[X > 0] >= -1e-11 * scale)
    assert np.all(g[X == 0] >= -1e-11 * scale)
    assert np.all(X >= 0)


def test_stop_rule_closed_form(orc):
    # One sweep with a huge eps_STOL stops at once; the reported step and norm
    # are ||(x1, y1) - (x0, y0)|| and ||(x0, y0)||.
    M, X0, Yt0 = small_problem(5)
    r = orc.anls(M, X0, Yt0, eps_stol=1e30, max_sweeps=10)
    assert r["sweeps"] == 1 and r["met"]
    d = np.sqrt(np.sum((r["X"] - X0) ** 2) + np.sum((r["Yt"] - Yt0) ** 2))
    nrm = np.sqrt(np.sum(X0 ** 2) + np.sum(Yt0 ** 2))
    assert r["step"] == pytest.approx(d, rel=1e-12)
    assert r["norm"] == pytest.approx(nrm, rel=1e-12)


def test_exact_sweeps_and_determinism(orc):
    M, X0, Yt0 = small_problem(6)
    a = orc.anls(M, X0, Yt0, exact_sweeps=7)
    b = orc.anls(M, X0, Yt0, exact_sweeps=7)
    assert a["sweeps"] == 7 and not a["met"]
    assert np.array_equal(a["X"], b["X"]) and np.array_equal(a["Yt"], b["Yt"])
    # sweeps compose: 3 then 4 equals 7
    c = orc.anls(M, X0, Yt0, exact_sweeps=3)
    d = orc.anls(M, c["X"], c["Yt"], exact_sweeps=4)
    assert np.array_equal(d["X"], a["X"]) and np.array_equal(d["Yt"], a["Yt"])


def test_thread_count_does_not_change_result(orc):
    M, X0, Yt0 = small_problem(7, n=300, m=40, k=5)
    t0 = orc.threads()
    try:
        orc.set_threads(1)
        a = orc.anls(M, X0, Yt0, exact_sweeps=5)
        orc.set_threads(max(2, t0))
        b = orc.anls(M, X0, Yt0, exact_sweeps=5)
    finally:
        orc.set_threads(t0)
    assert np.array_equal(a["X"], b["X"]) and np.array_equal(a["Yt"], b["Yt"])


def test_anls_fixed_point_at_convergence(orc):
    # Once the stop rule holds, one more sweep moves the point by at most
    # about eps_STOL (1 + ||(x, y)||).
    M, X0, Yt0 = small_problem(8, n=100, m=30, k=3)
    r = orc.anls(M, X0, Yt0, eps_stol=1e-10, max_sweeps=20000)
    assert r["met"]
    s = orc.anls(M, r["X"], r["Yt"], exact_sweeps=1)
    d = np.sqrt(np.sum((s["X"] - r["X"]) ** 2) + np.sum((s["Yt"] - r["Yt"]) ** 2))
    assert d <= 1e-9 * (1 + r["norm"])
