"""Hand-value pins for the oracle's step rules of the interior-point stage.

Every expected number below is worked out by hand in the comment beside it,
from the paper's definitions: the predictor probe and the centring rule of
eq. (8)-(9), the mu update and the exact-Hessian flag of Alg. 3 (Sec. IV),
the Armijo rule of eq. (13), the barrier merit function phi of Sec. III-A,
E(.;0) of eq. (10) with the stage-1 duals of Sec. V-A, and the transition
eq. (21)-(25) on a case with several rows, columns and components.  Each is
chosen so that a plausible slip (a square for the cube, tau = 0.9 in the
probe, < for <=, eta = 0, a per-component maximum, |graX| for max(graX, 0))
changes the result.
"""
import math

import numpy as np
import pytest


def test_affine_mu_hand_values(orc):
    # n = 1, m = 1, k = 2.
    #   dr = -r - (r/x) dx = [-0.5 + 1, -1 - 0.25] = [0.5, -1.25]
    #   ds = -s - (s/y) dy = [-0.25 - 0.125, -2 + 1] = [-0.375, -1]
    #   alpha1 (tau = 1) = min(1, 1/2, 1/0.5) = 0.5
    #   alpha2 (tau = 1) = min(1, 1/1.25, 0.25/0.375, 2/1) = 2/3
    #   x + a1 dx = [0, 4.5], r + a2 dr = [5/6, 1/6]
    #   y + a1 dy = [2.5, 0.75], s + a2 ds = [0, 4/3]
    #   mu_aff = (0 + 4.5/6 + 0 + 0.75 * 4/3) / 4 = 1.75 / 4 = 0.4375
    X = np.array([[1.0, 4.0]])
    Yt = np.array([[2.0, 1.0]])
    r = np.array([[0.5, 1.0]])
    s = np.array([[0.25, 2.0]])
    dxa = np.array([[-2.0, 1.0]])
    dya = np.array([[1.0, -0.5]])
    assert orc.affine_mu(X, Yt, r, s, dxa, dya) == pytest.approx(0.4375, rel=1e-15)
    # the average complementarity: (0.5 + 4 + 0.5 + 2) / 4 = 1.75
    assert orc.complementarity_avg(X, Yt, r, s) == pytest.approx(1.75, rel=1e-15)


def test_affine_mu_steps_to_the_boundary(orc):
    # n = m = k = 1: the tau = 1 steps reach the boundary of both pairs.
    #   dr = -0.5 - 0.5 * (-2) = 0.5,  ds = -0.25 - 0.125 = -0.375
    #   alpha1 = 1/2, alpha2 = 0.25/0.375 = 2/3
    #   (1 - 1)(0.5 + 1/3) + (2.5)(0.25 - 0.25) = 0 exactly.
    # With tau = 0.9 in the probe the result would be
    #   (0.1)(0.8) + (2.45)(0.025) = 0.14125, / 2 = 0.070625.
    X, Yt = np.array([[1.0]]), np.array([[2.0]])
    r, s = np.array([[0.5]]), np.array([[0.25]])
    assert orc.affine_mu(X, Yt, r, s, np.array([[-2.0]]), np.array([[1.0]])) == 0.0


def test_centring_rule_hand_values(orc):
    # sigma = min((mu_aff / avg)^3, 0.99), eq. (9)
    assert orc.centring(0.5, 1.0) == 0.125            # a square would give 0.25
    assert orc.centring(0.4375, 1.75) == 0.015625     # (1/4)^3
    assert orc.centring(3.0, 2.0) == 0.99             # capped
    assert orc.centring(-1e-17, 1.0) == 0.0           # rounding residue below 0 counts as 0
    assert orc.centring(0.0, 1.0) == 0.0


def test_mu_and_flag_update_hand_values(orc):
    # mu <- sigma * avg; flag = 1 exactly when sigma <= sigma_c (Sec. IV)
    assert orc.mu_flag_update(0.015625, 1.75, 0.01) == (0.02734375, 0)
    mu, flag = orc.mu_flag_update(0.01, 2.0, 0.01)
    assert mu == 0.02 and flag == 1                   # equality switches (<=, not <)
    assert orc.mu_flag_update(np.nextafter(0.01, 1.0), 2.0, 0.01)[1] == 0
    assert orc.mu_flag_update(0.0, 2.0, 0.01) == (0.0, 1)


def test_armijo_rejects_a_decrease_short_of_eta(orc):
    # phi(a) = (a - 1)^2, phi(0) = 1, slope -2, first trial a1 = 1.9.
    #   t = 0: phi(1.9) = 0.81 < 1 but 0.81 > 1 + 0.5 * 1.9 * (-2) = -0.9: rejected
    #   t = 1: phi(0.95) = 0.0025 <= 1 - 0.95 = 0.05: accepted
    # With eta = 0 the first trial would already pass.
    al, t, phi1, capped = orc.armijo(lambda a: (a - 1.0) ** 2, 1.0, 1.9, -2.0, 0.5, 60)
    assert (al, t, capped) == (0.95, 1, False)
    assert phi1 == pytest.approx(0.0025, rel=1e-12)
    al0, t0, _, _ = orc.armijo(lambda a: (a - 1.0) ** 2, 1.0, 1.9, -2.0, 0.0, 60)
    assert (al0, t0) == (1.9, 0)


def test_armijo_accepts_equality_and_caps(orc):
    # phi(a) = 1 - a with slope -1 and eta = 1 meets the rule with equality at
    # the first trial (<=, not <).
    al, t, _, capped = orc.armijo(lambda a: 1.0 - a, 1.0, 1.0, -1.0, 1.0, 60)
    assert (al, t, capped) == (1.0, 0, False)
    # a flat phi never passes: after max_backtracks = 3 halvings the last
    # trial, a1 / 8, is taken and flagged
    al, t, _, capped = orc.armijo(lambda a: 1.0, 1.0, 1.0, -1.0, 0.5, 3)
    assert (al, t, capped) == (0.125, 3, True)


def test_ipm_uses_the_pinned_rules(orc, monkeypatch):
    # the interior-point loop takes its step, centring and flag decisions from
    # the functions pinned above
    import oracle.ipm_oracle as io
    calls = {"armijo": 0, "centring": [], "update": []}
    real_armijo, real_centring, real_update = io.armijo, io.centring, io.mu_flag_update

    def armijo(*a):
        calls["armijo"] += 1
        return real_armijo(*a)

    def centring(mu_aff, avg):
        sig = real_centring(mu_aff, avg)
        calls["centring"].append(sig)
        return sig

    def update(sig, avg, sc):
        out = real_update(sig, avg, sc)
        calls["update"].append((sig, avg, out))
        return out
    monkeypatch.setattr(io, "armijo", armijo)
    monkeypatch.setattr(io, "centring", centring)
    monkeypatch.setattr(io, "mu_flag_update", update)
    rng = np.random.default_rng(3)
    X = rng.uniform(0.2, 1.0, (8, 2))
    Yt = rng.uniform(0.2, 1.0, (5, 2))
    M = X @ Yt.T + 0.05 * rng.standard_normal((8, 5))
    X1, Y1, r1, s1, mu1, rho1 = orc.transition(M, X, Yt, 1e-10)
    res = orc.ipm(M, X1, Y1, r1, s1, mu1, rho1, orc.IPMOptions(eps_tol=1e-10, max_inner=7))
    assert calls["armijo"] == res.inner == 7
    assert len(calls["centring"]) >= 2 and calls["update"]
    sig, avg, (mu, flag) = calls["update"][-1]
    assert mu == sig * avg and flag == int(sig <= 0.01)


def test_merit_hand_values(orc):
    # phi(x, y) = 1/2 ||XY - M||^2 - mu (sum log x + sum log y)
    # n = m = k = 1: R = 6 - 5 = 1, phi = 0.5 - 0.1 log 6
    assert orc.merit(np.array([[5.0]]), np.array([[2.0]]), np.array([[3.0]]), 0.1) == \
        pytest.approx(0.5 - 0.1 * math.log(6.0), rel=1e-15)
    # k = 2 with an exact fit: XY = 0.5 + 0.5 = 1 = M, so
    # phi = -0.5 (log 1 + log 2 + log 0.5 + log 0.25) = 0.5 log 4 = log 2
    assert orc.merit(np.array([[1.0]]), np.array([[1.0, 2.0]]), np.array([[0.5, 0.25]]), 0.5) == \
        pytest.approx(math.log(2.0), rel=1e-14)
    # outside the open orthant the barrier is +inf
    assert orc.merit(np.array([[1.0]]), np.array([[0.0]]), np.array([[1.0]]), 0.1) == np.inf


def test_kkt_error_anls_hand_values(orc):
    # E(.;0) with r = max(graX, 0), s = max(graY, 0) (Sec. V-A).
    # R = XY - M = 6 - 5 = 1; graX = R y = 3, graY = x R = 2; r = 3, s = 2;
    # gradient part 0, complementarity ||(3*2, 2*3)|| = 6 sqrt(2)
    X, Yt = np.array([[2.0]]), np.array([[3.0]])
    assert orc.kkt_error_anls(np.array([[5.0]]), X, Yt) == pytest.approx(6.0 * math.sqrt(2.0), rel=1e-15)
    # R = -1: graX = -3, graY = -2, r = s = 0: E = sqrt(9 + 4)
    assert orc.kkt_error_anls(np.array([[7.0]]), X, Yt) == pytest.approx(math.sqrt(13.0), rel=1e-15)
    # two rows of opposite residual sign: R = [1, -2]; graX = [1, -2],
    # graY = 1 - 2 = -1; r = [1, 0], s = 0; gradient part ||(0, -2, -1)|| =
    # sqrt(5), complementarity ||(1, 0, 0)|| = 1; E = sqrt(5)
    # (|graX| in place of max(graX, 0) would give sqrt(20))
    E = orc.kkt_error_anls(np.array([[0.0], [3.0]]), np.array([[1.0], [1.0]]), np.array([[1.0]]))
    assert E == pytest.approx(math.sqrt(5.0), rel=1e-15)


def test_transition_hand_example_several_components(orc):
    # X = [[1, 2], [3, 4]], Y = [[1, 2], [1, 1]] (Yt = Y^T), M = [[2, 4], [7, 12]]:
    #   XY = [[3, 4], [7, 10]], R = XY - M = [[1, 0], [0, -2]]
    #   graX = R Y^T = [[1, 1], [-4, -2]]       -> r = max |graX| = 4
    #   graY^T = R^T X = [[1, 2], [-6, -8]]     -> s = max |graY| = 8
    #   rho0 = 1e-6 * max(4, 2) = 4e-6: nothing is clamped
    #   mu = (4 * (1 + 2 + 3 + 4) + 8 * (1 + 1 + 2 + 1)) / (4 + 4) = 10
    # A per-component maximum would give r = [4, 2]; one maximum over both
    # gradients would give r = 8.
    X = np.array([[1.0, 2.0], [3.0, 4.0]])
    Yt = np.array([[1.0, 1.0], [2.0, 1.0]])
    M = np.array([[2.0, 4.0], [7.0, 12.0]])
    X1, Y1, r, s, mu, rho = orc.transition(M, X, Yt, 1e-8)
    assert np.array_equal(X1, X) and np.array_equal(Y1, Yt)
    assert np.all(r == 4.0) and np.all(s == 8.0)
    assert mu == 10.0 and rho == 1e-6


def test_transition_clamps_from_the_larger_factor_maximum(orc):
    # rho0 = 1e-6 * max(max X, max Y) on the point before clamping, eq. (22):
    # here max Y = 5 > max X = 1, so the zero entry of X becomes 5e-6.
    X = np.array([[1.0, 0.0]])
    Yt = np.array([[5.0, 1.0]])
    M = np.array([[4.0]])
    X1, Y1, _, _, _, _ = orc.transition(M, X, Yt, 1e-8)
    assert X1[0, 1] == pytest.approx(5e-6, rel=1e-15)
    assert X1[0, 0] == 1.0 and np.array_equal(Y1, Yt)
