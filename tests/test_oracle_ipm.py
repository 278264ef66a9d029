"""Pins for the oracle's transition and interior-point stage (Sec. III, IV).

The Newton direction is checked against a dense solve of the full 4-block
system eq. (11) (and of the exact-Hessian system, with the Hessian taken by
finite differences of the gradient), the gradients against finite differences
of f, the end point against the KKT conditions eq. (3) through scipy's
independent NNLS, and the objective against Table III of the paper.
"""
import os

import numpy as np
import pytest
from scipy.optimize import nnls as scipy_nnls

from paper_2101_08431_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(seed, n=6, m=4, k=2, near_fit=False):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.2, 1.0, (n, k))
    Yt = rng.uniform(0.2, 1.0, (m, k))
    M = X @ Yt.T + (0.01 if near_fit else 0.5) * rng.standard_normal((n, m))
    r = rng.uniform(0.1, 1.0, (n, k))
    s = rng.uniform(0.1, 1.0, (m, k))
    return M, X, Yt, r, s


def f_of(M, X, Yt):
    return 0.5 * np.sum((X @ Yt.T - M) ** 2)


def test_gradients_match_finite_differences(orc):
    M, X, Yt, _, _ = tiny(1)
    gx, gy, R = orc.gradients(M, X, Yt)
    h = 1e-6
    for (A, G) in ((X, gx), (Yt, gy)):
        for idx in np.ndindex(A.shape):
            A[idx] += h
            fp = f_of(M, X, Yt)
            A[idx] -= 2 * h
            fm = f_of(M, X, Yt)
            A[idx] += h
            assert G[idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-8)


def dense_hessian_fd(M, X, Yt):
    """Hessian of f in (x, y) = (vec(X^T), vec(Y)) by central differences of
    the gradient (the gradient itself is pinned above)."""
    import oracle
    n, k = X.shape
    m = Yt.shape[0]
    N = n * k + m * k
    H = np.zeros((N, N))
    h = 1e-5
    v = np.concatenate([X.ravel(), Yt.ravel()])

    def grad(v):
        gx, gy, _ = oracle.gradients(M, v[:n * k].reshape(n, k), v[n * k:].reshape(m, k))
        return np.concatenate([gx.ravel(), gy.ravel()])
    for q in range(N):
        e = np.zeros(N)
        e[q] = h
        H[:, q] = (grad(v + e) - grad(v - e)) / (2 * h)
    return 0.5 * (H + H.T)


def dense_gauss_newton(X, Yt):
    """J^T J for the residual XY - M, with J from its definition:
    d(XY)_ij / dX_ia = Y_aj, d(XY)_ij / dY_aj = X_ia."""
    n, k = X.shape
    m = Yt.shape[0]
    J = np.zeros((n * m, n * k + m * k))
    for i in range(n):
        for j in range(m):
            row = i * m + j
            J[row, i * k:(i + 1) * k] = Yt[j]
            J[row, n * k + j * k:n * k + (j + 1) * k] = X[i]
    return J.T @ J


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_direction_matches_dense_4block_system(orc, seed):
    # eq. (11) with Delta r and Delta s kept as unknowns, solved densely.
    M, X, Yt, r, s = tiny(seed)
    n, k = X.shape
    m = Yt.shape[0]
    mu, rho = 0.3, 0.02
    gx, gy, R = orc.gradients(M, X, Yt)
    dx, dy = orc.newton_direction(X, Yt, r, s, mu, rho, gx, gy, R, exact=False)
    nk, mk = n * k, m * k
    N = nk + mk
    A = np.zeros((2 * N, 2 * N))
    A[:N, :N] = dense_gauss_newton(X, Yt) + rho * np.eye(N)
    A[:N, N:] = -np.eye(N)
    A[N:, :N] = np.diag(np.concatenate([r.ravel(), s.ravel()]))
    A[N:, N:] = np.diag(np.concatenate([X.ravel(), Yt.ravel()]))
    z = np.concatenate([X.ravel(), Yt.ravel()])
    d = np.concatenate([r.ravel(), s.ravel()])
    rhs = np.concatenate([d - np.concatenate([gx.ravel(), gy.ravel()]), mu - d * z])
    sol = np.linalg.solve(A, rhs)
    np.testing.assert_allclose(dx.ravel(), sol[:nk], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dy.ravel(), sol[nk:N], rtol=1e-10, atol=1e-12)


def test_exact_direction_matches_fd_hessian(orc):
    # flag = 1: the Hessian of eq. (4)-(5) (blocks Q1, Q2 and C) equals the
    # true Hessian of f; compare the direction with one built from a finite
    # difference Hessian.
    M, X, Yt, r, s = tiny(4, near_fit=True)
    n, k = X.shape
    m = Yt.shape[0]
    mu, rho = 0.05, 1e-3
    gx, gy, R = orc.gradients(M, X, Yt)
    d = orc.newton_direction(X, Yt, r, s, mu, rho, gx, gy, R, exact=True)
    assert d is not None
    H = dense_hessian_fd(M, X, Yt)
    z = np.concatenate([X.ravel(), Yt.ravel()])
    dual = np.concatenate([r.ravel(), s.ravel()])
    B = H + rho * np.eye(len(z)) + np.diag(dual / z)
    g = np.concatenate([gx.ravel(), gy.ravel()]) - mu / z
    p = np.linalg.solve(B, -g)
    np.testing.assert_allclose(np.concatenate([d[0].ravel(), d[1].ravel()]), p, rtol=1e-6, atol=1e-8)


def test_exact_direction_reports_indefinite_schur(orc):
    # A large residual makes the exact Hessian indefinite; the Schur matrix then
    # has no Cholesky factor and the routine says so.
    rng = np.random.default_rng(9)
    X = rng.uniform(0.2, 1.0, (6, 2))
    Yt = rng.uniform(0.2, 1.0, (4, 2))
    M = X @ Yt.T + 25.0
    r = np.full_like(X, 1e-6)
    s = np.full_like(Yt, 1e-6)
    gx, gy, R = orc.gradients(M, X, Yt)
    assert orc.newton_direction(X, Yt, r, s, 1e-6, 1e-6, gx, gy, R, exact=True) is None
    assert orc.newton_direction(X, Yt, r, s, 1e-6, 1e-6, gx, gy, R, exact=False) is not None


def test_gauss_newton_direction_is_descent(orc):
    for seed in range(5):
        M, X, Yt, r, s = tiny(10 + seed, n=9, m=5, k=3)
        gx, gy, R = orc.gradients(M, X, Yt)
        mu = 0.1
        dx, dy = orc.newton_direction(X, Yt, r, s, mu, 1e-6, gx, gy, R)
        slope = np.sum(dx * (gx - mu / X)) + np.sum(dy * (gy - mu / Yt))
        assert slope < 0


def test_kkt_error_hand_values(orc):
    # n = m = k = 1: X = 2, Y = 3, r = 0.5, s = 0.25, graX = 1, graY = -1.
    X = np.array([[2.0]])
    Yt = np.array([[3.0]])
    r = np.array([[0.5]])
    s = np.array([[0.25]])
    E = orc.kkt_error(X, Yt, r, s, 0.1, np.array([[1.0]]), np.array([[-1.0]]))
    # gradient part sqrt(0.5^2 + 1.25^2); complementarity sqrt(0.9^2 + 0.65^2)
    assert E == pytest.approx(max(np.hypot(0.5, 1.25), np.hypot(0.9, 0.65)), rel=1e-15)


def test_kkt_error_zero_at_exact_factorisation(orc):
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, (7, 2))
    Yt = rng.uniform(0, 1, (5, 2))
    M = X @ Yt.T
    assert orc.kkt_error_anls(M, X, Yt) <= 1e-14


def test_step_max_hand_values(orc):
    v = np.array([1.0, 2.0, 4.0])
    dv = np.array([-1.0, 1.0, -8.0])
    # tau = 0.9: min(0.9 * 1 / 1, 0.9 * 4 / 8) = 0.45
    assert orc.step_max([(v, dv)], 0.9) == pytest.approx(0.45, rel=1e-15)
    assert orc.step_max([(v, dv)], 1.0) == pytest.approx(0.5, rel=1e-15)
    assert orc.step_max([(v, np.abs(dv))], 0.9) == 1.0


def test_transition_hand_example(orc):
    # M = [[4]], X = [[2]], Y = [[0]]: rho0 = 2e-6 clamps Y; the residual is
    # 4e-6 - 4, graX = (4e-6 - 4) * 2e-6, graY = 2 (4e-6 - 4).
    X, Yt, r, s, mu, rho = orc.transition(np.array([[4.0]]), np.array([[2.0]]),
                                          np.array([[0.0]]), 1e-8)
    y0 = 2e-6
    res = 2.0 * y0 - 4.0
    assert Yt[0, 0] == y0 and X[0, 0] == 2.0
    assert r[0, 0] == pytest.approx(abs(res * y0), rel=1e-15)
    assert s[0, 0] == pytest.approx(abs(2.0 * res), rel=1e-15)
    assert mu == pytest.approx((2.0 * r[0, 0] + y0 * s[0, 0]) / 2.0, rel=1e-15)
    assert rho == 1e-6


def test_two_stage_end_point_is_kkt(orc):
    # E(.;0) <= eps_TOL certifies eq. (3).  Independently: the end point is a
    # fixed point of both NNLS subproblems (scipy's NNLS).
    M, X0, Y0 = synth.make("pdf_200x50_k3", 1)
    res = orc.solve(M, X0, Y0.T.copy(), orc.IPMOptions(eps_tol=1e-10))
    assert res["converged"] and res["E0"] <= 1e-10
    X, Yt = res["X"], res["Yt"]
    assert np.all(X > 0) and np.all(Yt > 0)
    tol = 1e-6 * max(np.abs(X).max(), np.abs(Yt).max())
    for i in range(0, M.shape[0], 7):
        xs, _ = scipy_nnls(Yt, M[i, :])
        np.testing.assert_allclose(X[i], xs, atol=tol)
    for j in range(M.shape[1]):
        ys, _ = scipy_nnls(X, M[:, j])
        np.testing.assert_allclose(Yt[j], ys, atol=tol)


def test_merit_monotone_within_inner_loops(orc):
    M, X0, Y0 = synth.make("pdf_200x50_k3", 0)
    opts = orc.IPMOptions(eps_tol=1e-9, history=True)
    res = orc.solve(M, X0, Y0.T.copy(), opts)
    ip = res["ipm"]
    assert res["converged"]
    for outer in ip.phi_hist:
        for phi0, phi1 in outer:
            assert phi1 <= phi0 + 1e-12 * abs(phi0)


def test_separable_recovery(orc):
    # Noiseless separable data has a unique NMF up to scaling and permutation;
    # from a 10 % perturbation of the truth the two-stage method recovers it.
    n, m, k = 40, 20, 3
    M, xs, ys = synth.separable(n, m, k, 3)
    X0, Y0 = synth.perturbed_init(xs, ys, 3, 0.1)
    res = orc.solve(np.asarray(M), X0, Y0.T.copy(), orc.IPMOptions(eps_tol=1e-10))
    assert res["converged"]
    assert res["f"] <= 1e-14 * 0.5 * np.sum(np.asarray(M) ** 2)
    Xn, Ytn = orc.normalise(res["X"], res["Yt"])
    Xt, Ytt = orc.normalise(xs, ys.T)
    perm = [int(np.argmax(np.abs(Xn.T @ Xt[:, a]))) for a in range(k)]
    assert sorted(perm) == list(range(k))
    np.testing.assert_allclose(Xn[:, perm], Xt, atol=1e-6)
    np.testing.assert_allclose(Ytn[:, perm], Ytt, atol=1e-6 * np.abs(Ytt).max())


@pytest.mark.slow
def test_table3_objective(orc):
    # Table III: on U(0,1) data with noise 0.1 the 2-STAGE f for (2000, 100, 4)
    # is 954.230.  Our noise draw differs, so f agrees to within 2 %.
    rows = [tuple(float(t) for t in line.split()) for line in
            open(os.path.join(GOLDEN, "table3_synthetic_f.txt")) if line.strip() and not line.startswith("#")]
    table = {(int(a), int(b), int(c)): f for a, b, c, f in rows}
    n, m, k = 2000, 100, 4
    M, _, _ = synth.uniform(n, m, k, seed=11)
    X0, Y0 = synth.random_init(n, m, k, 11, float(np.linalg.norm(M)))
    res = orc.solve(np.asarray(M), X0, Y0.T.copy(), orc.IPMOptions(eps_tol=1e-6))
    assert res["converged"]
    assert abs(res["f"] / table[(n, m, k)] - 1.0) < 0.02
