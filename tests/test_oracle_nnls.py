"""Pins for the oracle's Lawson-Hanson NNLS (the subproblem eq. (2) of Sec. II).

The subproblem min 1/2 ||C x - d||^2, x >= 0 with C of full column rank is
strictly convex, so its minimiser is the unique point that satisfies the KKT
conditions.  These tests check the oracle against that definition by brute
force over all 2^k passive sets, against scipy's independent NNLS routine, and
against closed forms.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import nnls as scipy_nnls


def brute_force(G, b):
    """Enumerate every passive set P; return the unique one whose solution
    z_P = G_PP^-1 b_P is positive and whose dual w = b - G z is <= 0 off P."""
    k = len(b)
    hits = []
    for r in range(k + 1):
        for P in itertools.combinations(range(k), r):
            P = list(P)
            z = np.zeros(k)
            if P:
                z[P] = np.linalg.solve(G[np.ix_(P, P)], b[P])
                if np.any(z[P] <= 0):
                    continue
            w = b - G @ z
            off = [a for a in range(k) if a not in P]
            if off and np.any(w[off] > 0):
                continue
            hits.append((z, sum(1 << a for a in P)))
    return hits


def margin_problem(rng, k, rows=None):
    """Random (G, b) whose solution has a clear margin: passive entries
    >= 1e-6 ||x|| and active duals <= -1e-6 ||b||, so the active set is
    decided far from rounding."""
    rows = rows or 3 * k + 2
    while True:
        C = rng.standard_normal((rows, k))
        d = rng.standard_normal(rows)
        G, b = C.T @ C, C.T @ d
        hits = brute_force(G, b)
        if len(hits) != 1:
            continue
        z, P = hits[0]
        w = b - G @ z
        pas = [a for a in range(k) if P >> a & 1]
        act = [a for a in range(k) if not P >> a & 1]
        if pas and np.min(z[pas]) < 1e-6 * np.linalg.norm(z):
            continue
        if act and np.max(w[act]) > -1e-6 * np.linalg.norm(b):
            continue
        return C, d, G, b, z, P


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 8])
def test_nnls_matches_brute_force(orc, k):
    rng = np.random.default_rng(100 + k)
    for _ in range(60 if k <= 6 else 15):
        _, _, G, b, z, P = margin_problem(rng, k)
        x, mask, st, _ = orc.nnls(G, b)
        assert st == 0
        assert mask == P, "active set must be bit-exact"
        assert np.all(x[[a for a in range(k) if not P >> a & 1]] == 0.0)
        np.testing.assert_allclose(x, z, rtol=1e-11, atol=1e-13 * max(1.0, np.abs(z).max()))


@pytest.mark.parametrize("k", [2, 5, 10, 16])
def test_nnls_matches_scipy(orc, k):
    rng = np.random.default_rng(7 + k)
    for _ in range(100):
        C = rng.standard_normal((2 * k + 3, k))
        d = rng.standard_normal(2 * k + 3)
        xs, _ = scipy_nnls(C, d)
        x, mask, st, _ = orc.nnls(C.T @ C, C.T @ d)
        assert st == 0
        np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-10 * max(1.0, np.abs(xs).max()))


def test_nnls_k1_closed_form(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        g = rng.uniform(0.1, 5.0)
        b = rng.standard_normal()
        x, mask, st, _ = orc.nnls(np.array([[g]]), np.array([b]))
        assert x[0] == pytest.approx(max(0.0, b / g), rel=1e-15)
        assert mask == (1 if b > 0 else 0)


def test_nnls_hand_example(orc):
    # G = [[2, 1], [1, 2]], b = (3, -1): the unconstrained solution (7/3, -5/3)
    # is infeasible; with x2 = 0 the first row gives x1 = 3/2, and the dual
    # w2 = -1 - 3/2 = -5/2 < 0 confirms optimality.
    x, mask, st, _ = orc.nnls(np.array([[2.0, 1.0], [1.0, 2.0]]), np.array([3.0, -1.0]))
    assert st == 0 and mask == 0b01
    np.testing.assert_allclose(x, [1.5, 0.0], rtol=1e-15)


def test_nnls_diagonal_and_nonpositive(orc):
    G = np.diag([1.0, 2.0, 4.0, 8.0])
    b = np.array([-1.0, 3.0, 0.0, 2.0])
    x, mask, st, _ = orc.nnls(G, b)
    np.testing.assert_allclose(x, [0.0, 1.5, 0.0, 0.25], rtol=1e-15)
    assert mask == 0b1010
    x, mask, st, _ = orc.nnls(G, -np.abs(b) - 1.0)
    assert np.all(x == 0.0) and mask == 0


def test_nnls_dead_component(orc):
    # A zero column of C gives a zero row and column in G and b_a = 0:
    # that variable stays at zero and the rest is the reduced problem.
    rng = np.random.default_rng(5)
    C = rng.standard_normal((9, 4))
    C[:, 2] = 0.0
    d = rng.standard_normal(9)
    x, mask, st, _ = orc.nnls(C.T @ C, C.T @ d)
    xs, _ = scipy_nnls(np.delete(C, 2, axis=1), d)
    assert x[2] == 0.0 and not (mask >> 2 & 1)
    np.testing.assert_allclose(np.delete(x, 2), xs, rtol=1e-9, atol=1e-12)


def test_nnls_zero_problem(orc):
    x, mask, st, _ = orc.nnls(np.zeros((3, 3)), np.zeros(3))
    assert st == 0 and mask == 0 and np.all(x == 0.0)


def test_nnls_kkt_on_many_random(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        k = int(rng.integers(1, 12))
        C = rng.uniform(0, 1, (20, k))
        d = rng.uniform(-0.5, 1.0, 20)
        G, b = C.T @ C, C.T @ d
        x, mask, st, _ = orc.nnls(G, b)
        w = b - G @ x
        scale = np.abs(b).max() + np.abs(G).max() * np.abs(x).sum()
        assert np.all(x >= 0)
        assert np.all(w <= 1e-12 * scale)                  # dual feasibility
        assert np.all(np.abs(w[x > 0]) <= 1e-11 * scale)   # stationarity on P
