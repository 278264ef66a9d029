"""Writes the oracle's two-stage end points on the paper's synthetic benchmark.

Calls only the CPU oracle (``oracle/``) and the seeded input generator.  The
workload is the synthetic set of Sec. V-D (Table III): X*, Y* ~ U(0, 1),
Gaussian noise sigma = 0.1, M clipped at 0, n = 2000.  For each (m, k) below,
seed 0: stage 1 (Alg. 1) to the Sec. IV rule with eps_STOL = 1e-6, then the
transition and Alg. 3 to E(.;0) <= 1e-8.  Stored per case (compressed .npz,
float64): the stage-1 end point, the final iterate, f, E(.;0) and counts.

    python tests/golden/make_synthetic_golden.py
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

CASES = [(50, 3), (100, 4)]
EPS_TOL = 1e-8


def main():
    for m, k in CASES:
        spec = dict(kind="uniform", n=2000, m=m, k=k, sigma=0.1)
        M, X0, Y0 = synth.make(spec, 0)
        M = np.asarray(M)
        t0 = time.time()
        opts = oracle.IPMOptions(eps_tol=EPS_TOL, eps_stol=1e-6, max_inner=20000, max_outer=20000)
        st1 = oracle.anls(M, X0, Y0.T.copy(), eps_stol=opts.eps_stol, max_sweeps=opts.max_anls_sweeps)
        X, Yt, r, s, mu, rho = oracle.transition(M, st1["X"], st1["Yt"], opts.eps_tol, opts.rho0_factor, opts.rho)
        res = oracle.ipm(M, X, Yt, r, s, mu, rho, opts)
        f = oracle.objective(M, res.X, res.Yt)
        print(f"m={m} k={k}: {st1['sweeps']} sweeps, {res.inner} iterations, converged {res.converged}, "
              f"E0 {res.E0:.2e}, f {f:.10e}, {time.time() - t0:.1f} s", flush=True)
        out = os.path.join(HERE, f"synthetic_2000x{m}_k{k}_seed0.npz")
        np.savez_compressed(out, eps_tol=EPS_TOL, sweeps=st1["sweeps"], X1=st1["X"], Yt1=st1["Yt"],
                            converged=res.converged, E0=res.E0, f=f, inner=res.inner, X=res.X, Yt=res.Yt)
        print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
