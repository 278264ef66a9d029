"""FP64 numpy oracle for the transition and the interior-point stage.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows, in the paper's order and notation:
  * Sec. III-A  the KKT system eq. (3), the Newton system eq. (4)-(5), the
    primal-dual system with the Gauss-Newton Hessian plus rho I, eq. (11), and
    its reduced form eq. (12); the fraction-to-boundary rule eq. (7); the
    predictor probe eq. (8)-(9); the error function eq. (10); the barrier merit
    function phi and the Armijo rule eq. (13) of Alg. 2;
  * Sec. III-B  the solution of eq. (12) by the block Cholesky factor
    Q1bar = P^T P and the Schur complement eq. (20), with C P^-1 formed densely
    as printed;
  * Sec. IV     the transition eq. (21)-(25), the exact-Hessian switch
    eq. (26)-(27) and Alg. 3.

Arrays: X (n, k) row i = X_i, so X.ravel() = x = vec(X^T); Yt (m, k) row j = Y_j,
so Yt.ravel() = y = vec(Y); r (n, k) and s (m, k) likewise.

Readings where the paper is silent, ambiguous or garbled:
  * norms in E are Euclidean; the Diag(Y) in eq. (10) is read as Diag(y);
  * the upper-right block of eq. (26) is read as Cbar^T (symmetric), and eq. (27)
    as [Q1 + rho I, C^T; C, Q2 + rho I];
  * eq. (23) uses the gradients at the clamped point; r and s get separate
    maxima, each floored at eps_TOL;
  * rho of eq. (25) is the paper's eps_TOL, 1e-6, and stays 1e-6 when a
    tighter stop tolerance is asked for (a smaller rho leaves the Gauss-Newton
    matrix all but singular along the scaling direction (X D, D^-1 Y), where f
    is flat, and the Armijo search then stalls);
  * in mu <- sigma mu (Alg. 2, Alg. 3) the mu on the right is the current
    average complementarity (x^T r + y^T s)/(nk + mk), the quantity sigma is
    measured against in eq. (9), as in the predictor heuristic the paper takes
    from Nocedal and Wright;
  * the predictor solves eq. (11) with Cbar and mu = 0;
  * "Repeat until" tests sit at the loop head; the inner loop also ends once
    E(.;0) <= eps_TOL, and after at most ``inner_cap`` (3) iterations at one mu.
    The cap is needed because for n != m the barrier problem has no stationary
    point: summing the stationarity conditions of component a over the rows of
    X and over the columns of Y gives n mu = m mu, so at fixed mu the iterates
    drift along the scaling direction and E(.;mu) <= mu is not reached;
  * at most 60 halvings in the Armijo search, after which the last trial step
    is taken and counted;
  * with flag = 1 a failed Cholesky factorisation of the Schur matrix counts
    like a non-descent direction: flag <- 0 and the step is recomputed with
    Cbar.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class IPMOptions:
    eps_tol: float = 1e-6          # Sec. V-A
    eps_stol: float = 1e-6         # Sec. IV stop rule; value not given in the paper
    tau: float = 0.9               # Sec. III-A
    eta: float = 0.5               # Alg. 3
    sigma_c: float = 0.01          # Sec. IV
    rho0_factor: float = 1e-6      # eq. (22)
    rho: float = 1e-6              # eq. (25): the paper's eps_TOL
    inner_cap: int = 3             # iterations at one mu before the mu update
    exact_hessian_switch: bool = True
    max_anls_sweeps: int = 5000
    max_outer: int = 200
    max_inner: int = 1000          # total inner iterations over the whole stage
    max_backtracks: int = 60
    history: bool = False
    snapshots: tuple = ()          # E(.;0) levels at which to keep a copy of the iterate


def gradients(M, X, Yt):
    """graX = (XY - M) Y^T as (n, k), graY = X^T (XY - M) as (m, k) (eq. (4)),
    and the residual R = XY - M."""
    R = X @ Yt.T - M
    return R @ Yt, R.T @ X, R


def kkt_error(X, Yt, r, s, mu, graX, graY):
    """E(x, y, r, s; mu), eq. (10)."""
    g = np.concatenate([(graX - r).ravel(), (graY - s).ravel()])
    c = np.concatenate([(r * X).ravel(), (s * Yt).ravel()]) - mu
    return max(float(np.linalg.norm(g)), float(np.linalg.norm(c)))


def kkt_error_anls(M, X, Yt):
    """E(.; 0) for a point without duals, with r = max(graX, 0) and
    s = max(graY, 0) (Sec. V-A)."""
    gx, gy, _ = gradients(M, X, Yt)
    return kkt_error(X, Yt, np.maximum(gx, 0.0), np.maximum(gy, 0.0), 0.0, gx, gy)


def merit(M, X, Yt, mu):
    """Barrier merit phi(x, y) of Sec. III-A; +inf outside the open orthant."""
    if np.any(X <= 0) or np.any(Yt <= 0):
        return np.inf
    R = X @ Yt.T - M
    return 0.5 * float(np.sum(R * R)) - mu * float(np.sum(np.log(X))) - mu * float(np.sum(np.log(Yt)))


def transition(M, X, Yt, eps_tol, rho0_factor=1e-6, rho=1e-6):
    """Stage transition, eq. (21)-(25).  Returns (X, Yt, r, s, mu, rho)."""
    rho0 = rho0_factor * max(float(X.max()), float(Yt.max()))
    X = np.maximum(X, rho0)
    Yt = np.maximum(Yt, rho0)
    gx, gy, _ = gradients(M, X, Yt)
    rv = max(float(np.abs(gx).max()), eps_tol)
    sv = max(float(np.abs(gy).max()), eps_tol)
    r = np.full_like(X, rv)
    s = np.full_like(Yt, sv)
    n, k = X.shape
    m = Yt.shape[0]
    mu = (float(np.sum(X * r)) + float(np.sum(Yt * s))) / (m * k + n * k)
    return X, Yt, r, s, mu, rho


def _block_diag(B):
    nb, k, _ = B.shape
    D = np.zeros((nb * k, nb * k))
    for q in range(nb):
        D[q * k:(q + 1) * k, q * k:(q + 1) * k] = B[q]
    return D


def newton_direction(X, Yt, r, s, mu, rho, graX, graY, R, exact=False):
    """(dx, dy) from eq. (12) by the route of Sec. III-B, or None when the
    Schur matrix of eq. (20) has no Cholesky factor.

    exact=False uses Cbar (Gauss-Newton, eq. (11)); exact=True uses C of eq. (5),
    i.e. block (j, i) = X_i^T Y_j^T + (XY - M)_ij I."""
    n, k = X.shape
    m = Yt.shape[0]
    eye = np.eye(k)
    b1 = -(graX - mu / X)                       # -grad_x phi
    b2 = -(graY - mu / Yt)                      # -grad_y phi
    Q1 = (Yt.T @ Yt)[None, :, :] + rho * eye[None] + (r / X)[:, :, None] * eye[None]
    Q2 = (X.T @ X)[None, :, :] + rho * eye[None] + (s / Yt)[:, :, None] * eye[None]
    L1 = np.linalg.cholesky(Q1)                 # Q1bar_i = L_i L_i^T, P_i = L_i^T
    Pinv = np.linalg.inv(np.transpose(L1, (0, 2, 1)))
    Cb = np.einsum('ia,jb->jaib', X, Yt)        # block (j, i), entry (a, b) = X_ia Y_bj
    if exact:
        for a in range(k):
            Cb[:, a, :, a] += R.T
    W = np.einsum('jaib,ibc->jaic', Cb, Pinv).reshape(m * k, n * k)   # Cbar P^-1
    S = _block_diag(Q2) - W @ W.T
    PTb1 = np.einsum('iba,ib->ia', Pinv, b1)    # P^-T b1, block by block
    rhs = b2.ravel() - W @ PTb1.ravel()
    try:
        Ls = np.linalg.cholesky(S)
    except np.linalg.LinAlgError:
        return None
    dy = np.linalg.solve(Ls.T, np.linalg.solve(Ls, rhs))
    t = (PTb1.ravel() - W.T @ dy).reshape(n, k)
    dx = np.einsum('iab,ib->ia', Pinv, t)
    return dx, dy.reshape(m, k)


def step_max(pairs, tau):
    """Largest alpha in (0, 1] with v + alpha dv >= (1 - tau) v for every (v, dv)
    pair, eq. (7)."""
    a = 1.0
    for v, dv in pairs:
        neg = dv < 0
        if np.any(neg):
            a = min(a, float(np.min(-tau * v[neg] / dv[neg])))
    return a


def complementarity_avg(X, Yt, r, s):
    """(x^T r + y^T s) / (nk + mk): the average complementarity that eq. (9)
    measures mu_aff against."""
    N = X.size + Yt.size
    return (float(np.sum(X * r)) + float(np.sum(Yt * s))) / N


def affine_mu(X, Yt, r, s, dxa, dya):
    """mu_aff of eq. (8)-(9) for the predictor direction (dxa, dya) of the
    mu = 0 system: the dual parts follow eq. (11) with mu = 0,
    dr = -r - (r / x) dx, and the step lengths are those of eq. (7) with
    tau = 1 (the largest steps that keep the point in the closed orthant)."""
    dra = -r - (r / X) * dxa
    dsa = -s - (s / Yt) * dya
    a1a = step_max([(X, dxa), (Yt, dya)], 1.0)
    a2a = step_max([(r, dra), (s, dsa)], 1.0)
    N = X.size + Yt.size
    return (float(np.sum((X + a1a * dxa) * (r + a2a * dra)))
            + float(np.sum((Yt + a1a * dya) * (s + a2a * dsa)))) / N


def centring(mu_aff, avg):
    """sigma = min{(mu_aff / avg)^3, 0.99}, eq. (9).  mu_aff is a
    complementarity of points in the closed orthant, so it is >= 0 in exact
    arithmetic; a rounding residue below 0 from the step to the boundary
    counts as 0."""
    return min((max(mu_aff, 0.0) / avg) ** 3, 0.99)


def mu_flag_update(sigma, avg, sigma_c):
    """The update of Alg. 3 after the predictor: mu <- sigma * avg and the
    exact-Hessian flag, set exactly when sigma <= sigma_c (Sec. IV)."""
    return sigma * avg, (1 if sigma <= sigma_c else 0)


def armijo(phi, phi0, a1, slope, eta, max_backtracks):
    """Backtracking of Alg. 2 / Alg. 3, eq. (13): the first t = 0, 1, ... with
    phi(a1 / 2^t) <= phi0 + eta (a1 / 2^t) slope.  After ``max_backtracks``
    halvings the last trial is taken.  Returns (alpha, t, phi(alpha), capped)."""
    t = 0
    while True:
        al = a1 / (2.0 ** t)
        phi1 = phi(al)
        if phi1 <= phi0 + eta * al * slope:
            return al, t, phi1, False
        if t >= max_backtracks:
            return al, t, phi1, True
        t += 1


@dataclass
class IPMResult:
    X: np.ndarray
    Yt: np.ndarray
    r: np.ndarray
    s: np.ndarray
    mu: float
    flag: int
    E0: float
    outer: int
    inner: int
    converged: bool
    backtrack_cap_hits: int = 0
    exact_steps: int = 0
    fallbacks: int = 0
    phi_hist: list = field(default_factory=list)
    E0_hist: list = field(default_factory=list)
    snapshots: dict = field(default_factory=dict)


def ipm(M, X, Yt, r, s, mu, rho, opts: IPMOptions):
    """Interior-point stage of Alg. 3 from a strictly interior point."""
    flag = 0
    gx, gy, R = gradients(M, X, Yt)
    E0 = kkt_error(X, Yt, r, s, 0.0, gx, gy)
    outer = inner = caps = exact_steps = fallbacks = 0
    phis, e0s = [], []
    snaps = {}
    while E0 > opts.eps_tol and outer < opts.max_outer and inner < opts.max_inner:
        outer += 1
        eps_mu = mu
        phis.append([])
        at_mu = 0
        while (kkt_error(X, Yt, r, s, mu, gx, gy) > eps_mu and E0 > opts.eps_tol
               and inner < opts.max_inner and at_mu < opts.inner_cap):
            inner += 1
            at_mu += 1
            gphi_x = gx - mu / X
            gphi_y = gy - mu / Yt
            d = None
            if flag == 1 and opts.exact_hessian_switch:
                d = newton_direction(X, Yt, r, s, mu, rho, gx, gy, R, exact=True)
                if d is not None:
                    slope = float(np.sum(d[0] * gphi_x) + np.sum(d[1] * gphi_y))
                    if slope >= 0:
                        d = None
                if d is None:
                    flag = 0
                    fallbacks += 1
                else:
                    exact_steps += 1
            if d is None:
                d = newton_direction(X, Yt, r, s, mu, rho, gx, gy, R, exact=False)
                if d is None:
                    raise FloatingPointError("Schur matrix of the Gauss-Newton system is not SPD")
            dx, dy = d
            dr = mu / X - r - (r / X) * dx
            ds = mu / Yt - s - (s / Yt) * dy
            a1 = step_max([(X, dx), (Yt, dy)], opts.tau)
            a2 = step_max([(r, dr), (s, ds)], opts.tau)
            slope = float(np.sum(dx * gphi_x) + np.sum(dy * gphi_y))
            phi0 = merit(M, X, Yt, mu)
            al, _, phi1, capped = armijo(lambda a: merit(M, X + a * dx, Yt + a * dy, mu), phi0, a1, slope,
                                         opts.eta, opts.max_backtracks)
            caps += int(capped)
            X = X + al * dx
            Yt = Yt + al * dy
            r = r + a2 * dr
            s = s + a2 * ds
            if opts.history:
                phis[-1].append((phi0, phi1))
            gx, gy, R = gradients(M, X, Yt)
            E0 = kkt_error(X, Yt, r, s, 0.0, gx, gy)
            e0s.append(E0)
            for lev in opts.snapshots:
                if E0 <= lev and lev not in snaps:
                    snaps[lev] = dict(X=X.copy(), Yt=Yt.copy(), r=r.copy(), s=s.copy(), E0=E0, inner=inner,
                                      outer=outer)
        if E0 <= opts.eps_tol:
            break
        # predictor (affine scaling) probe, eq. (8)-(9)
        d = newton_direction(X, Yt, r, s, 0.0, rho, gx, gy, R, exact=False)
        if d is None:
            raise FloatingPointError("Schur matrix of the predictor system is not SPD")
        mu_aff = affine_mu(X, Yt, r, s, d[0], d[1])
        avg = complementarity_avg(X, Yt, r, s)
        sigma = centring(mu_aff, avg)
        mu, flag = mu_flag_update(sigma, avg, opts.sigma_c)
    return IPMResult(X=X, Yt=Yt, r=r, s=s, mu=mu, flag=flag, E0=E0, outer=outer, inner=inner,
                     converged=E0 <= opts.eps_tol, backtrack_cap_hits=caps,
                     exact_steps=exact_steps, fallbacks=fallbacks, phi_hist=phis, E0_hist=e0s,
                     snapshots=snaps)


def two_stage(M, X0, Yt0, opts: IPMOptions = None, anls_fn=None):
    """Alg. 3: ANLS (stage 1) to the Sec. IV step rule, the transition, then the
    interior-point stage to E(.;0) <= eps_TOL.  ``anls_fn`` is the stage-1
    routine (the C oracle's ``anls``)."""
    if opts is None:
        opts = IPMOptions()
    M = np.asarray(M, dtype=np.float64)
    st1 = anls_fn(M, X0, Yt0, eps_stol=opts.eps_stol, max_sweeps=opts.max_anls_sweeps)
    X, Yt, r, s, mu, rho = transition(M, st1["X"], st1["Yt"], opts.eps_tol, opts.rho0_factor,
                                      opts.rho)
    res = ipm(M, X, Yt, r, s, mu, rho, opts)
    return dict(stage1=st1, ipm=res, X=res.X, Yt=res.Yt,
                f=0.5 * float(np.sum((res.X @ res.Yt.T - M) ** 2)), E0=res.E0,
                converged=res.converged)


def normalise(X, Yt):
    """Scale every column of X to unit Euclidean norm and move the scale into
    the matching row of Y (column of Yt).  Removes the scaling freedom of NMF
    so end points can be compared."""
    c = np.linalg.norm(X, axis=0)
    c = np.where(c > 0, c, 1.0)
    return X / c[None, :], Yt * c[None, :]
