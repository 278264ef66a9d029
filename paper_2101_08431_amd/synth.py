"""Seeded synthetic inputs for streaming NMF, min 1/2 ||XY - M||_F^2, X, Y >= 0.

This module only draws data.  It holds none of the factorisation's arithmetic,
so both the GPU path and the CPU oracle may take their inputs from it.

Layouts handed out (all float64, numpy):
  * ``M``  shape (n, m), Fortran order: column j (one time instant) is
    contiguous, i.e. element (i, j) sits at offset j*n + i.  This is the
    column-major layout the C ABI takes with ``ldm = n``.
  * ``X0`` shape (n, k), ``Y0`` shape (k, m), C order.

Workloads
---------
``pdf_like``   stands in for the streaming pair-distribution-function data of
               Sec. V-B (the AgMOR set, which is not available here): every
               column of X* is a sum of 4-8 Gaussian peaks on r in [0, 20]
               (heights U(0.2, 1), widths U(0.05, 0.3)); every column of Y* is a
               vector of smooth logistic phase fractions in time that sum to 1.
               M = max(X* Y* + noise, 0).
``uniform``    the synthetic set of Sec. V-D: X*, Y* ~ U(0, 1), Gaussian noise
               with standard deviation 0.1, negative entries of M set to 0.
``separable``  noiseless M = X* Y* where X* holds k rows and Y* holds k columns
               that are scaled unit vectors; the factorisation is then unique up
               to scaling and permutation (used to check exact recovery).

Draw order (fixed, so a seed names one input): peaks per column of X* in
column order (count, then centres, heights, widths); then the k-1 logistic
centres and the common width; then the noise matrix in row-major (n, m) order.
The random initial point uses its own stream, seeded ``seed + 1000003``.
"""
from __future__ import annotations

import numpy as np

INIT_SEED_OFFSET = 1000003


def _pdf_factors(rng, n, m_horizon, k):
    r = np.linspace(0.0, 20.0, n)
    xs = np.zeros((n, k))
    for p in range(k):
        npk = int(rng.integers(4, 9))
        c = rng.uniform(0.0, 20.0, npk)
        h = rng.uniform(0.2, 1.0, npk)
        w = rng.uniform(0.05, 0.3, npk)
        for q in range(npk):
            xs[:, p] += h[q] * np.exp(-((r - c[q]) ** 2) / (2.0 * w[q] ** 2))
    t = np.linspace(0.0, 1.0, m_horizon) if m_horizon > 1 else np.zeros(1)
    cen = np.sort(rng.uniform(0.15, 0.85, k - 1))
    om = rng.uniform(0.03, 0.10)
    logi = [1.0 / (1.0 + np.exp(-(t - c) / om)) for c in cen]
    ys = np.zeros((k, m_horizon))
    if k == 1:
        ys[0] = 1.0
    else:
        ys[0] = 1.0 - logi[0]
        for p in range(1, k - 1):
            ys[p] = logi[p - 1] - logi[p]
        ys[k - 1] = logi[k - 2]
    return xs, ys


def pdf_like(n, m, k, seed, sigma=1e-3, sigma_relative=False, m_horizon=None):
    """PDF-like streaming data.  Returns (M, X*, Y*).

    ``sigma`` is the noise standard deviation; with ``sigma_relative`` it is
    scaled by max(X* Y*).  ``m_horizon`` >= m fixes the time grid of a stream
    whose later columns arrive afterwards: the first m columns are returned and
    a larger ``m`` with the same horizon extends them unchanged.
    """
    mh = m if m_horizon is None else int(m_horizon)
    if mh < m:
        raise ValueError("m_horizon must be >= m")
    rng = np.random.default_rng(seed)
    xs, ys = _pdf_factors(rng, n, mh, k)
    clean = xs @ ys
    s = sigma * (clean.max() if sigma_relative else 1.0)
    noise = rng.standard_normal((n, mh))
    mfull = np.maximum(clean + s * noise, 0.0)
    return np.asfortranarray(mfull[:, :m]), xs, ys[:, :m].copy()


def uniform(n, m, k, seed, sigma=0.1):
    """The synthetic workload of Sec. V-D.  Returns (M, X*, Y*)."""
    rng = np.random.default_rng(seed)
    xs = rng.uniform(0.0, 1.0, (n, k))
    ys = rng.uniform(0.0, 1.0, (k, m))
    noise = rng.standard_normal((n, m))
    mm = np.maximum(xs @ ys + sigma * noise, 0.0)
    return np.asfortranarray(mm), xs, ys


def separable(n, m, k, seed):
    """Noiseless separable data.  Returns (M, X*, Y*).

    Rows 0..k-1 of X* are d_a e_a and columns 0..k-1 of Y* are g_a e_a with
    d, g ~ U(1, 2); all other entries ~ U(0, 1).
    """
    if n < k or m < k:
        raise ValueError("separable data needs n >= k and m >= k")
    rng = np.random.default_rng(seed)
    xs = rng.uniform(0.0, 1.0, (n, k))
    ys = rng.uniform(0.0, 1.0, (k, m))
    xs[:k, :] = np.diag(rng.uniform(1.0, 2.0, k))
    ys[:, :k] = np.diag(rng.uniform(1.0, 2.0, k))
    return np.asfortranarray(xs @ ys), xs, ys


def random_init(n, m, k, seed, m_target_norm):
    """Random non-negative start X0, Y0 ~ U(0, 1) from stream ``seed + 1000003``,
    scaled by one common factor so that ||X0 Y0||_F equals ``m_target_norm``."""
    rng = np.random.default_rng(seed + INIT_SEED_OFFSET)
    x0 = rng.uniform(0.0, 1.0, (n, k))
    y0 = rng.uniform(0.0, 1.0, (k, m))
    cur = np.linalg.norm(x0 @ y0)
    if cur > 0 and m_target_norm > 0:
        s = np.sqrt(m_target_norm / cur)
        x0 *= s
        y0 *= s
    return x0, y0


def perturbed_init(xs, ys, seed, rel=0.1):
    """Start near a known factorisation: each entry times (1 + rel*U(-1, 1))."""
    rng = np.random.default_rng(seed + INIT_SEED_OFFSET)
    x0 = xs * (1.0 + rel * rng.uniform(-1.0, 1.0, xs.shape))
    y0 = ys * (1.0 + rel * rng.uniform(-1.0, 1.0, ys.shape))
    return np.maximum(x0, 0.0), np.maximum(y0, 0.0)


# Named workloads (n, m, k) with their noise rule.
WORKLOADS = {
    "pdf_200x50_k3": dict(kind="pdf", n=200, m=50, k=3, sigma=1e-3, sigma_relative=False),
    "pdf_3000x500_k5": dict(kind="pdf", n=3000, m=500, k=5, sigma=1e-3, sigma_relative=True),
    "pdf_10000x2000_k10": dict(kind="pdf", n=10000, m=2000, k=10, sigma=1e-3, sigma_relative=True),
}


def make(name_or_spec, seed):
    """Build (M, X0, Y0) for a named workload with the given seed."""
    spec = WORKLOADS[name_or_spec] if isinstance(name_or_spec, str) else dict(name_or_spec)
    n, m, k = spec["n"], spec["m"], spec["k"]
    kind = spec.get("kind", "pdf")
    if kind == "pdf":
        mm, _, _ = pdf_like(n, m, k, seed, sigma=spec.get("sigma", 1e-3),
                            sigma_relative=spec.get("sigma_relative", False))
    elif kind == "uniform":
        mm, _, _ = uniform(n, m, k, seed, sigma=spec.get("sigma", 0.1))
    elif kind == "separable":
        mm, _, _ = separable(n, m, k, seed)
    else:
        raise ValueError(kind)
    x0, y0 = random_init(n, m, k, seed, float(np.linalg.norm(mm)))
    return mm, x0, y0


# ------------------------------------------------------------------ serving
def serving_streams(count=64, big_every=5, small=(2000, 4), big=(8000, 8)):
    """(n, k) of each stream: every ``big_every``-th stream (index 0 mod
    big_every) is ``big``, the others ``small``."""
    return [big if (s % big_every == 0) else small for s in range(count)]


def serving_trace(streams, rate, seconds, seed=7):
    """Open-loop Poisson arrivals at ``rate`` requests/s in total over
    ``seconds``; each request picks a stream uniformly.  Returns a list of
    (arrival time in s, stream index), sorted by time."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        out.append((t, int(rng.integers(0, streams))))
    return out


def serving_stream_data(n, k, m0, add, requests, seed, sigma=1e-3):
    """One stream's data: the first ``m0`` columns and ``requests`` blocks of
    ``add`` new columns, all from one PDF-like stream whose time grid spans
    m0 + add * requests instants.  Returns (M0, [blocks], X0, Y0), every block
    (n, add) in Fortran order, X0, Y0 a random start for M0."""
    mh = m0 + add * requests
    mfull, _, _ = pdf_like(n, mh, k, seed, sigma=sigma, sigma_relative=True, m_horizon=mh)
    M0 = np.asfortranarray(mfull[:, :m0])
    blocks = [np.asfortranarray(mfull[:, m0 + add * q: m0 + add * (q + 1)]) for q in range(requests)]
    x0, y0 = random_init(n, m0, k, seed, float(np.linalg.norm(M0)))
    return M0, blocks, x0, y0
