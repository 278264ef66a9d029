"""Writes the oracle's first interior-point iteration at 10000 x 2000 x 10 as a fixture.

Calls only the CPU oracle (``oracle/``) and the seeded input generator.  For
the PDF-like workload of that size, seed 0: exactly 20 stage-1 sweeps (Alg. 1)
from the seeded start, the transition eq. (21)-(25) with eps_TOL = 1e-8, then
one inner iteration of Alg. 3 (Gauss-Newton direction of eq. (11) through the
Schur complement eq. (20) of order mk = 20000, step rules eq. (7), Armijo
search eq. (13)).  Stored (compressed .npz, float64): the iterate and duals
after that iteration, the step count and the barrier parameter.

    python tests/golden/make_ipm_first_golden.py

needs about 45 GB of memory (the oracle forms Cbar P^-1 densely, 16 GB) and
several minutes of BLAS time.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_08431_amd import synth  # noqa: E402

NAME, SEED, SWEEPS, EPS_TOL = "pdf_10000x2000_k10", 0, 20, 1e-8


def main():
    M, X0, Y0 = synth.make(NAME, SEED)
    M = np.asarray(M)
    t0 = time.time()
    st1 = oracle.anls(M, X0, Y0.T.copy(), exact_sweeps=SWEEPS)
    print(f"stage 1: {SWEEPS} sweeps, {time.time() - t0:.1f} s", flush=True)
    opts = oracle.IPMOptions(eps_tol=EPS_TOL, max_inner=1)
    X, Yt, r, s, mu, rho = oracle.transition(M, st1["X"], st1["Yt"], opts.eps_tol, opts.rho0_factor, opts.rho)
    res = oracle.ipm(M, X, Yt, r, s, mu, rho, opts)
    print(f"one iteration: inner {res.inner}, {time.time() - t0:.1f} s", flush=True)
    out = os.path.join(HERE, f"ipm1_{NAME}_seed{SEED}.npz")
    np.savez_compressed(out, sweeps=SWEEPS, eps_tol=EPS_TOL, inner=res.inner, X=res.X, Yt=res.Yt, r=res.r, s=res.s)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
