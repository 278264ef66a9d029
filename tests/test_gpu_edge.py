"""Degenerate stage-1 inputs on the GPU against the CPU oracle.

* exactly tied multipliers at a cold start with a non-singular Gram matrix
  (the first index of largest w enters; the result is unique);
* a singular Gram matrix (two equal rows of Y0): the minimisers of the X-half
  are not unique, so the unique fitted product X Y0 is compared and the KKT
  conditions of both halves are checked on the GPU's iterate;
* a dead component: a zero row of Y0 gives G_aa = 0, which never enters;
* duplicate columns of X0: only the warm start sees X0 (the X-half solves X
  from Y0), so the iterates are the oracle's cold-start ones;
* M with negative entries (eq. (1) is defined for any M).

Bar (unique cases): factors within 1e-8 of the largest entry after the same
sweeps, passive sets bit-exact, every entry finite and >= 0."""
import numpy as np
import pytest

from paper_2101_08431_amd import synth

pytestmark = pytest.mark.gpu

REL = 1e-8


def run_gpu(M, k, X0, Y0, sweeps):
    from paper_2101_08431_amd import NMF, default_options
    ctx = NMF(np.asfortranarray(M), k, X0, Y0,
              options=default_options(eps_stol=-1.0, max_anls_sweeps=1 << 30, with_ipm=0))
    ctx.anls_step(sweeps)
    X, Y = ctx.factors()
    xm, ym = ctx.masks()
    ctx.close()
    return X, Y, xm, ym


def check(orc, M, k, X0, Y0, sweeps):
    X, Y, xm, ym = run_gpu(M, k, X0, Y0, sweeps)
    ref = orc.anls(np.asfortranarray(M), X0, Y0.T.copy(), exact_sweeps=sweeps)
    assert np.isfinite(X).all() and np.isfinite(Y).all()
    assert (X >= 0).all() and (Y >= 0).all()
    scale = max(np.abs(ref["X"]).max(), np.abs(ref["Yt"]).max())
    err = max(np.abs(X - ref["X"]).max(), np.abs(Y.T - ref["Yt"]).max()) / scale
    assert err <= REL, err
    assert np.array_equal(xm, ref["xmask"]) and np.array_equal(ym, ref["ymask"])
    return X, Y, ref


def nnls_kkt_ok(G, B, X, rel=1e-9):
    """KKT of min 1/2 x^T G x - b^T x, x >= 0 for every row x of X (b the
    matching row of B): x >= 0, w = b - G x <= tol, |w_a| <= tol where x_a > 0."""
    W = B - X @ G.T
    tol = rel * (np.abs(B) + X @ np.abs(G).T).max(axis=1, keepdims=True)
    return bool((X >= 0).all() and (W <= tol).all() and (np.abs(W[X > 0]) <= np.broadcast_to(tol, X.shape)[X > 0]).all())


def test_tied_w_full_rank(orc):
    # X0 = 0 makes the first X-half start cold, so its first entering index
    # is chosen among exactly tied multipliers: rows 0 and 1 of Y0 are
    # orthogonal with equal norms, and row i of M is c_i v with v = (2, 2, 1,
    # 1, ...) (equal sums over even and odd columns), so b_0 = b_1 and
    # G_00 = G_11 exactly (small integers, exact in FP64).  G_Y is
    # non-singular and component 2 (y = (0, 0, 1, 1, ...)) has a clear
    # negative multiplier, so the X-half's minimiser and passive sets are
    # unique: compared with the oracle entry by entry and bit-exactly.  The
    # new X has equal columns 0 and 1, so the Y-half's minimisers are not
    # unique: its KKT conditions are checked on the GPU's iterate.
    n, m, k = 70, 40, 3
    rng = np.random.default_rng(6)
    v = np.tile([2.0, 2.0, 1.0, 1.0], m // 4)
    M = rng.integers(1, 5, (n, 1)).astype(float) * v[None, :]
    Y0 = np.zeros((k, m))
    Y0[0, 0::2] = 1.0
    Y0[1, 1::2] = 1.0
    Y0[2] = np.tile([0.0, 0.0, 1.0, 1.0], m // 4)
    X0 = np.zeros((n, k))
    print("case tied w, full-rank G, one sweep", flush=True)
    X, Y, xm, _ = run_gpu(M, k, X0, Y0, 1)
    ref = orc.anls(np.asfortranarray(M), X0, Y0.T.copy(), exact_sweeps=1)
    assert np.isfinite(X).all() and np.isfinite(Y).all()
    assert np.abs(X - ref["X"]).max() <= 1e-8 * np.abs(ref["X"]).max()
    assert np.array_equal(xm, ref["xmask"]) and (xm == 3).all()
    assert nnls_kkt_ok(X.T @ X, (X.T @ M).T, Y.T)


def test_singular_gram_valid(orc):
    # two equal rows of Y0 make G_Y singular: the X-half's minimisers are not
    # unique, but the fitted rows X Y0 are (the projection of a row of M onto
    # the cone spanned by the rows of Y0).  Compared: X Y0 with the oracle's;
    # checked: the KKT conditions of the X-half (given Y0) and of the Y-half
    # (given the new X) on the GPU's own iterate.
    rng = np.random.default_rng(5)
    n, m, k = 70, 40, 3
    M = rng.integers(0, 5, (n, m)).astype(float)
    Y0 = rng.integers(0, 4, (k, m)).astype(float)
    Y0[1] = Y0[0]
    X0 = rng.integers(0, 4, (n, k)).astype(float)
    print("case singular G_Y (equal rows of Y0), one sweep", flush=True)
    X, Y, _, _ = run_gpu(M, k, X0, Y0, 1)
    ref = orc.anls(np.asfortranarray(M), X0, Y0.T.copy(), exact_sweeps=1)
    assert np.isfinite(X).all() and np.isfinite(Y).all()
    fit, fit_ref = X @ Y0, ref["X"] @ Y0
    assert np.abs(fit - fit_ref).max() <= 1e-8 * np.abs(fit_ref).max()
    assert nnls_kkt_ok(Y0 @ Y0.T, M @ Y0.T, X)
    assert nnls_kkt_ok(X.T @ X, (X.T @ M).T, Y.T)


def test_dead_component(orc):
    M, X0, Y0 = synth.make(dict(kind="pdf", n=260, m=90, k=4, sigma=1e-3, sigma_relative=True), 8)
    Y0 = Y0.copy()
    Y0[2] = 0.0
    print("case dead component (zero row of Y0)", flush=True)
    X, Y, _ = check(orc, M, 4, X0, Y0, 4)
    assert (X[:, 2] == 0).all() and (Y[2] == 0).all()


def test_duplicate_columns_of_x0(orc):
    M, X0, Y0 = synth.make(dict(kind="pdf", n=333, m=71, k=5, sigma=1e-3, sigma_relative=True), 9)
    X0 = X0.copy()
    X0[:, 3] = X0[:, 1]
    print("case duplicate columns of X0", flush=True)
    check(orc, M, 5, X0, Y0, 5)


def test_negative_entries_of_m(orc):
    M, X0, Y0 = synth.make(dict(kind="pdf", n=300, m=80, k=4, sigma=1e-2, sigma_relative=False), 4)
    M = M - 0.1 * M.mean()
    assert (M < 0).any()
    print("case M with negative entries", flush=True)
    check(orc, M, 4, X0, Y0, 5)
