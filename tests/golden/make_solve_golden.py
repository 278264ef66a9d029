"""Writes the oracle's two-stage end point of a full-size solve as a fixture.

Calls only the CPU oracle (``oracle/``) and the seeded input generator.  For
the PDF-like workload of the given size and seed: stage 1 (Alg. 1) to the
Sec. IV step rule with eps_STOL = 1e-6, the transition eq. (21)-(25), then the
interior-point stage of Alg. 3 to E(.;0) <= eps_tol.  Stored (compressed
.npz, float64): the stage-1 end point, the iterate where E(.;0) first drops to
1e-8, and the final iterate with its duals, objective and counts.

    python tests/golden/make_solve_golden.py pdf_3000x500_k5 0 1e-10

takes about half an hour on 8 cores (one Newton direction of the 2500 x 2500
Schur system is about 2 s in numpy).
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


def main(name, seed, eps_tol):
    M, X0, Y0 = synth.make(name, seed)
    M = np.asarray(M)
    opts = oracle.IPMOptions(eps_tol=eps_tol, eps_stol=1e-6, max_inner=20000, max_outer=20000,
                             snapshots=(1e-8,))
    t0 = time.time()
    st1 = oracle.anls(M, X0, Y0.T.copy(), eps_stol=opts.eps_stol, max_sweeps=opts.max_anls_sweeps)
    print(f"stage 1: {st1['sweeps']} sweeps, {time.time() - t0:.1f} s", flush=True)
    X, Yt, r, s, mu, rho = oracle.transition(M, st1["X"], st1["Yt"], opts.eps_tol, opts.rho0_factor, opts.rho)
    res = oracle.ipm(M, X, Yt, r, s, mu, rho, opts)
    f = oracle.objective(M, res.X, res.Yt)
    print(f"stage 2: converged {res.converged}, E0 {res.E0:.3e}, {res.inner} iterations, {res.outer} mu "
          f"updates, f {f:.15e}, {time.time() - t0:.1f} s", flush=True)
    snap = res.snapshots.get(1e-8)
    out = os.path.join(HERE, f"solve_{name}_seed{seed}.npz")
    np.savez_compressed(
        out, eps_tol=eps_tol, eps_stol=opts.eps_stol, sweeps=st1["sweeps"], X1=st1["X"], Yt1=st1["Yt"],
        converged=res.converged, E0=res.E0, f=f, inner=res.inner, outer=res.outer, X=res.X, Yt=res.Yt,
        r=res.r, s=res.s, exact_steps=res.exact_steps, fallbacks=res.fallbacks,
        X_1e8=snap["X"] if snap else np.zeros(0), Yt_1e8=snap["Yt"] if snap else np.zeros(0),
        inner_1e8=snap["inner"] if snap else -1, E0_1e8=snap["E0"] if snap else -1.0)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), float(sys.argv[3]))
