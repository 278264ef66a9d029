"""FP64 CPU oracle for two-stage streaming NMF (Gu, Du, Billinge).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package imports nothing from the product package.

* ``anls_oracle.c``  the ANLS stage (Sec. II, Alg. 1) in plain C, loaded here
  through ctypes: cold-started Lawson-Hanson NNLS, the two half-steps, the
  objective and the Sec. IV stop rule.
* ``ipm_oracle.py``  the transition and the interior-point stage (Sec. III,
  Sec. IV, Alg. 2 and Alg. 3) in numpy.

Array conventions (vec rules under eq. (3)): X is (n, k) with row i = X_i;
``Yt`` is (m, k) with row j = Y_j, the j-th column of Y; M is (n, m) and is
passed to C in column-major order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "anls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_anls.so")
_lib = None


def build(force=True):
    """Compile the C part of the oracle with gcc (plain -O2, OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint32)
        ip = ctypes.POINTER(ctypes.c_int)
        i64 = ctypes.c_int64
        L.orc_nnls.argtypes = [ctypes.c_int, dp, dp, dp, up, ip]
        L.orc_nnls.restype = ctypes.c_int
        L.orc_half_x.argtypes = [i64, i64, ctypes.c_int, dp, i64, dp, dp, up]
        L.orc_half_x.restype = ctypes.c_int
        L.orc_half_y.argtypes = [i64, i64, ctypes.c_int, dp, i64, dp, dp, up]
        L.orc_half_y.restype = ctypes.c_int
        L.orc_objective.argtypes = [i64, i64, ctypes.c_int, dp, i64, dp, dp]
        L.orc_objective.restype = ctypes.c_double
        L.orc_anls.argtypes = [i64, i64, ctypes.c_int, dp, i64, dp, dp, ctypes.c_double,
                               ctypes.c_int, up, up, dp]
        L.orc_anls.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_kmax.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _colmajor(M):
    M = np.asarray(M, dtype=np.float64)
    return np.asfortranarray(M)


def threads():
    return int(lib().orc_threads())


def set_threads(t):
    lib().orc_set_threads(int(t))


def nnls(G, b):
    """Cold-start Lawson-Hanson: argmin 1/2 x^T G x - b^T x, x >= 0.

    Returns (x, passive_mask, status, n_solves)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    k = b.shape[0]
    x = np.zeros(k)
    P = np.zeros(1, dtype=np.uint32)
    ns = ctypes.c_int(0)
    st = lib().orc_nnls(k, _dp(G), _dp(b), _dp(x), _up(P), ctypes.byref(ns))
    return x, int(P[0]), int(st), int(ns.value)


def half_x(M, X, Yt):
    """X-half of Alg. 1.  Returns (X_new, masks, n_failed)."""
    Mc = _colmajor(M)
    n, m = Mc.shape
    k = X.shape[1]
    Xn = np.ascontiguousarray(X, dtype=np.float64).copy()
    Yc = np.ascontiguousarray(Yt, dtype=np.float64)
    masks = np.zeros(n, dtype=np.uint32)
    bad = lib().orc_half_x(n, m, k, _dp(Mc), n, _dp(Xn), _dp(Yc), _up(masks))
    return Xn, masks, bad


def half_y(M, X, Yt):
    """Y-half of Alg. 1.  Returns (Yt_new, masks, n_failed)."""
    Mc = _colmajor(M)
    n, m = Mc.shape
    k = X.shape[1]
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    Yn = np.ascontiguousarray(Yt, dtype=np.float64).copy()
    masks = np.zeros(m, dtype=np.uint32)
    bad = lib().orc_half_y(n, m, k, _dp(Mc), n, _dp(Xc), _dp(Yn), _up(masks))
    return Yn, masks, bad


def objective(M, X, Yt):
    """1/2 ||X Y - M||_F^2 computed from the residual."""
    Mc = _colmajor(M)
    n, m = Mc.shape
    k = X.shape[1]
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    Yc = np.ascontiguousarray(Yt, dtype=np.float64)
    return float(lib().orc_objective(n, m, k, _dp(Mc), n, _dp(Xc), _dp(Yc)))


def anls(M, X0, Yt0, eps_stol=1e-6, max_sweeps=1000, exact_sweeps=None):
    """Alg. 1 from (X0, Yt0).  With ``exact_sweeps`` runs exactly that many
    sweeps (no stop rule).  Returns dict(X, Yt, xmask, ymask, sweeps, met,
    step, norm, failed)."""
    Mc = _colmajor(M)
    n, m = Mc.shape
    k = X0.shape[1]
    X = np.ascontiguousarray(X0, dtype=np.float64).copy()
    Yt = np.ascontiguousarray(Yt0, dtype=np.float64).copy()
    xm = np.zeros(n, dtype=np.uint32)
    ym = np.zeros(m, dtype=np.uint32)
    st = np.zeros(5)
    if exact_sweeps is not None:
        eps, cap = -1.0, int(exact_sweeps)
    else:
        eps, cap = float(eps_stol), int(max_sweeps)
    lib().orc_anls(n, m, k, _dp(Mc), n, _dp(X), _dp(Yt), eps, cap, _up(xm), _up(ym), _dp(st))
    return dict(X=X, Yt=Yt, xmask=xm, ymask=ym, sweeps=int(st[0]), met=bool(st[1]),
                step=float(st[2]), norm=float(st[3]), failed=int(st[4]))


from .ipm_oracle import (  # noqa: E402
    IPMOptions, gradients, kkt_error, kkt_error_anls, merit, transition, newton_direction,
    step_max, ipm, two_stage, normalise, complementarity_avg, affine_mu, centring, mu_flag_update, armijo,
)


def solve(M, X0, Yt0, opts=None):
    """Alg. 3 end to end: the C stage 1 followed by the numpy stage 2."""
    return two_stage(M, X0, Yt0, opts, anls_fn=anls)
