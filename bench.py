#!/usr/bin/env python3
"""Benchmark: column NNLS solves/s of the ANLS stage on one MI355X.

Headline workload: PDF-like streaming data, n = 3000 rows, m = 500 time
columns, rank k = 5, noise 1e-3 * max(X* Y*), seed 0 (a synthetic stand-in for
the streaming PDF data of Sec. V-B).  A timed step is one ANLS sweep (Alg. 1):
the X-half (B_X = M Y^T, then one warm-started NNLS per row) and the Y-half
(B_Y = X^T M, one NNLS per column), i.e. n + m column NNLS solves, replayed
from a captured HIP graph.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  Besides the headline fields:
  roofline      the dominant stage-1 kernel; per-kernel device times come from
                HIP events around each launch on the library's stream
  full_solve    Alg. 3 (ANLS, transition, interior point) to E(.;0) <= 1e-8 on
                four seeds of the headline workload
  precision     sweep time and error against the FP64 oracle of the FP32 and
                split-BF16 Gram forms on n = 10000, m = 2000, k = 10
  batching      256 uneven problems (n ~ U[500, 4000], m ~ U[100, 1000],
                k in 2..8): batched graph-replayed sweeps vs the plain
                per-problem launches
  cpu_baseline  the FP64 CPU oracle timed on a bounded number of sweeps of the
                headline workload on the host cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "column NNLS solves/s + full-solve time at KKT ≤1e-8; serving p50/p99 latency"
WORKLOAD = "pdf_3000x500_k5"


def algorithmic_bytes(n, m, k):
    """Bytes each stage-1 step must move at minimum per launch.

    k_xstream: read M (8nm) and Y (8km), write B_X (8nk).
    k_xnnls:   read B_X and X (16nk) and the row masks (4n), write X (8nk) and
               the masks (4n).
    k_ystream: read M (8nm) and X (8nk), write B_Y (8km).
    k_ynnls:   read B_Y and Y (16km), masks (4m), write Y (8km), masks (4m)."""
    return (8 * n * m + 8 * k * m + 8 * n * k,
            24 * n * k + 8 * n,
            8 * n * m + 8 * n * k + 8 * k * m,
            24 * k * m + 8 * m)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_ctx(M, X0, Y0, k, **opt):
    import numpy as np
    import torch
    from paper_2101_08431_amd import NMF, default_options
    base = dict(eps_stol=-1.0, max_anls_sweeps=1 << 30, with_ipm=0)
    base.update(opt)
    Md = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
    return NMF(Md, k, torch.from_numpy(X0).cuda(), torch.from_numpy(Y0).cuda(), options=default_options(**base))


def time_graph_sweeps(ctx, steps, warmup):
    """ms per sweep of graph-replayed sweeps (a batch of one problem: the
    batch form's table-driven kernels), the wall time of the timed replay, and
    ms per sweep of the same batch form launched eagerly (which separates the
    cost of the batch kernels from that of graph replay)."""
    import torch
    from paper_2101_08431_amd import Batch
    b = Batch([ctx])
    b.step(warmup, graph=True)
    b.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(b.stream)
    b.step(steps, graph=True)
    e1.record(b.stream)
    b.sync()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    dev = e0.elapsed_time(e1)
    b.step(warmup, graph=False)
    b.sync()
    e0.record(b.stream)
    b.step(steps, graph=False)
    e1.record(b.stream)
    b.sync()
    torch.cuda.synchronize()
    dev_eager = e0.elapsed_time(e1)
    b.close()
    return dev / steps, wall, dev_eager / steps


def time_eager_sweeps(ctx, steps, warmup):
    import torch
    ctx.anls_step(warmup, report=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    ctx.anls_step(steps, report=False)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measured_traffic(kernel, shape, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE scaled by a plain copy
    of known size), or None when there is none for this launch shape or the
    stage-1 kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    src = os.path.join(ROOT, "paper_2101_08431_amd", "csrc", "anls.hip")
    try:
        lines = open(path).read().splitlines()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    recorded = [ln.split()[2] for ln in lines if ln.startswith("source_sha256 anls.hip ")]
    if not recorded or recorded[0] != digest:
        return None
    want = f"{shape[0]},{shape[1]}"
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "traffic" and f[1] == kernel and f[2] == want:
            return float(f[3])
    return None


HEADLINE_SHAPES = [(8, 3), (8, 4), (8, 6), (4, 4), (4, 6), (11, 6)]


def roofline(ctx, n, m, k, shape, workload, sweeps=100):
    """Per-kernel device times from the library's event profiler and the
    algorithmic bytes of each kernel; shape is the launch plan (x splits,
    y splits, X one kernel, Y one kernel).  A half run as one kernel
    (k_xfused / k_yfused) moves the bytes of both of its steps."""
    ms = ctx.anls_profile(sweeps)
    by = algorithmic_bytes(n, m, k)
    per = {}
    if shape[2]:
        per["k_xfused"] = (ms[0] + ms[1], by[0] + by[1])
    else:
        per["k_xstream"], per["k_xnnls"] = (ms[0], by[0]), (ms[1], by[1])
    if shape[3]:
        per["k_yfused"] = (ms[2] + ms[3], by[2] + by[3])
    else:
        per["k_ystream"], per["k_ynnls"] = (ms[2], by[2]), (ms[3], by[3])
    per = {name: {"ms": t, "bytes": b, "GBs": b / (t * 1e-3) / 1e9} for name, (t, b) in per.items()}
    dom = max(per, key=lambda q: per[q]["ms"])
    ach = per[dom]["GBs"]
    # the whole sweep: every kernel's algorithmic bytes over the summed kernel times
    sweep_bytes = sum(v["bytes"] for v in per.values())
    sweep_ms = sum(v["ms"] for v in per.values())
    sweep_gbs = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(dom, shape, workload),
            "bytes_per_launch": per[dom]["bytes"], "launch_plan": list(shape), "per_kernel": per,
            "sweep": {"bytes": sweep_bytes, "ms": sweep_ms, "achieved": sweep_gbs, "frac": sweep_gbs / HBM_PEAK_GBS}}


def full_solve(name, seeds, tol, cap, mixed=0):
    import torch
    from paper_2101_08431_amd import NMF, default_options, synth
    from paper_2101_08431_amd._lib import NMFError
    out = []
    for seed in seeds:
        M, X0, Y0 = synth.make(name, seed)
        ctx = NMF(M, X0.shape[1], X0, Y0, options=default_options(eps_tol=tol, max_ipm_iters=cap))
        ctx.set_ipm_precision(mixed, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        note = None
        try:
            st, rep = ctx.solve()
        except NMFError as e:
            # a numerical breakdown (the Gauss-Newton Schur matrix stopped
            # factoring): reported with the iterate's state, not hidden
            st, note = e.status, str(e)
            rep = ctx.report()
        torch.cuda.synchronize()
        log(f"full solve seed {seed}: status {st}, E0 {rep['E0']:.2e}")
        row = {"seed": seed, "ms": (time.perf_counter() - t0) * 1e3, "status": int(st), "converged": st == 1,
               "E0": rep["E0"], "f": rep["f"], "sweeps": rep["sweeps"], "ipm_iters": rep["ipm_iters"],
               "exact_steps": rep["exact_steps"], "mu": rep["mu"],
               "ms_stage1": rep["ms_stage1"], "ms_stage2": rep["ms_stage2"]}
        if note:
            row["breakdown"] = note
        out.append(row)
        ctx.close()
    import statistics
    conv = [r["ms"] for r in out if r["converged"]]
    return {"workload": name, "tol": tol, "ipm_cap": cap, "mixed_precision": mixed, "runs": out,
            "converged": f"{len(conv)}/{len(out)}",
            "median_ms_converged": statistics.median(conv) if conv else None,
            "max_ms_converged": max(conv) if conv else None}


FP64_PEAK_TFS = 78.6


def ipm_section(name="pdf_3000x500_k5", seed=1, iters=10, sweeps=300, mixed=0):
    """Stage-2 timing (Alg. 3 inner iterations: direction, line search,
    update): the seed's problem after `sweeps` stage-1 sweeps, the transition
    and one iteration untimed, then `iters` iterations with the dense steps
    event-timed (nmf_ipm_profile), and the same number again untimed-per-step
    for the plain wall time per iteration.  Roofline entries for the
    Gauss-Newton Schur formation (eq. (20)) and the Cholesky factorisation of
    the Schur matrix against the FP64 peak."""
    import torch
    from paper_2101_08431_amd import NMF, default_options, synth
    M, X0, Y0 = synth.make(name, seed)
    n, m = M.shape
    k = X0.shape[1]
    ctx = NMF(M, k, X0, Y0, options=default_options(eps_tol=1e-8, eps_stol=-1.0, max_anls_sweeps=1 << 30))
    ctx.set_ipm_precision(mixed, 2)
    ctx.anls_step(sweeps, report=False)
    ctx.ipm_step(1)
    st, ms, cnt = ctx.ipm_profile(iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep = ctx.ipm_step(iters)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / max(1, iters)
    ctx.close()
    N = m * k
    nl = k * (k + 1) // 2
    gn_flop = n * (m * (m + 1) // 2) * 2 * (k + nl)     # c_ijl (k) and the k(k+1)/2 accumulations, j >= l
    chol_flop = N ** 3 / 3
    ex_flop = (N * (N + 1) // 2) * n * k * 2            # sum_i V_i^T V_i, lower triangle
    def tfs(f, t):
        return f / (t * 1e-3) / 1e12 if t > 0 else None
    out = {"workload": name, "seed": seed, "stage1_sweeps": sweeps, "iterations": iters, "mixed_precision": mixed,
           "ms_per_iteration": wall, "ms_per_iteration_profiled": ms[4], "schur_order": N,
           "E0_after": rep["E0"],
           "dense_steps_ms": {"gauss_newton_schur": ms[0], "exact_schur": ms[1], "cholesky": ms[2],
                              "triangular_solve_pair": ms[3]},
           "dense_steps_count": {"gauss_newton_schur": cnt[0], "exact_schur": cnt[1], "cholesky": cnt[2],
                                 "triangular_solve_pair": cnt[3], "inner_iterations": cnt[4]},
           "flop": {"gauss_newton_schur": gn_flop, "exact_schur": ex_flop, "cholesky": chol_flop}}
    out["roofline"] = {
        "gauss_newton_schur": {"kernel": "k_schur_gn (+ k_xx, k_schur_reduce)", "bound": "mfma",
                               "achieved": tfs(gn_flop, ms[0]), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                               "frac": (tfs(gn_flop, ms[0]) or 0.0) / FP64_PEAK_TFS},
        "cholesky": {"kernel": "k_chol_step x NT (+ k_pad_identity)", "bound": "mfma",
                     "achieved": tfs(chol_flop, ms[2]), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": (tfs(chol_flop, ms[2]) or 0.0) / FP64_PEAK_TFS},
    }
    if cnt[1]:
        # the FP32 form runs on FP32 matrix cores (157.3 TFLOP/s dense)
        pk = 157.3 if mixed else FP64_PEAK_TFS
        out["roofline"]["exact_schur"] = {"kernel": "k_vgen + k_syrk_v (+ k_syrk_reduce, k_linv, k_residual_rows)", "bound": "mfma",
                                          "dtype": "f32" if mixed else "f64",
                                          "achieved": tfs(ex_flop, ms[1]), "peak": pk,
                                          "unit": "TFLOP/s", "frac": (tfs(ex_flop, ms[1]) or 0.0) / pk}
    return out


def mixed_section():
    """Mixed-precision interior point (exact-Hessian Schur formation on FP32
    matrix cores, FP64 refinement): the profiled iterations of ipm_section in
    both precisions, and full solves to E(.;0) <= 1e-8 of seed 0 (few
    exact-Hessian steps) and seed 7 (mostly exact-Hessian steps) in both."""
    out = {"ipm_fp64": ipm_section(mixed=0), "ipm_mixed": ipm_section(mixed=1)}
    for mixed in (0, 1):
        out[f"solve_{'mixed' if mixed else 'fp64'}"] = full_solve("pdf_3000x500_k5", (0, 7), 1e-8, 5000, mixed)
    return out


def ipm_large_section(iters=3):
    """Stage 2 at n = 10000, m = 2000, k = 10 (Schur order 20000, S of 3.2 GB):
    the oracle's 20 stage-1 sweeps as the start, the transition and `iters`
    profiled iterations; the first iteration is compared with the oracle's
    (tests/golden/ipm1_pdf_10000x2000_k10_seed0.npz, written by an oracle-only
    script) when that file is present."""
    import numpy as np
    import oracle
    from paper_2101_08431_amd import synth
    name = "pdf_10000x2000_k10"
    M, X0, Y0 = synth.make(name, 0)
    M = np.asarray(M)
    n, m = M.shape
    k = X0.shape[1]
    st1 = oracle.anls(M, X0, Y0.T.copy(), exact_sweeps=20)
    from paper_2101_08431_amd import NMF, default_options
    ctx = NMF(np.asfortranarray(M), k, np.ascontiguousarray(st1["X"]), np.ascontiguousarray(st1["Yt"].T),
              options=default_options(eps_tol=1e-8, eps_stol=-1.0, max_anls_sweeps=1 << 30))
    out = {"workload": name, "schur_order": m * k, "schur_bytes": 8 * (m * k) ** 2}
    ctx.ipm_step(1)
    golden = os.path.join(ROOT, "tests", "golden", f"ipm1_{name}_seed0.npz")
    if os.path.exists(golden):
        g = np.load(golden)
        X, Y = ctx.factors()
        R, S = ctx.duals()
        sc = max(np.abs(g["X"]).max(), np.abs(g["Yt"]).max())
        out["first_iteration_error_vs_oracle"] = {
            "factors": float(max(np.abs(X - g["X"]).max(), np.abs(Y.T - g["Yt"]).max()) / sc),
            "duals": float(max(np.abs(R - g["r"]).max() / np.abs(g["r"]).max(),
                               np.abs(S.T - g["s"]).max() / np.abs(g["s"]).max()))}
    st, ms, cnt = ctx.ipm_profile(iters)
    ctx.close()
    N = m * k
    nl = k * (k + 1) // 2
    gn_flop = n * (m * (m + 1) // 2) * 2 * (k + nl)
    chol_flop = N ** 3 / 3
    out.update({"iterations": cnt[4], "ms_per_iteration": ms[4],
                "dense_steps_ms": {"gauss_newton_schur": ms[0], "exact_schur": ms[1], "cholesky": ms[2],
                                   "triangular_solve_pair": ms[3]},
                "roofline": {"gauss_newton_schur_frac": gn_flop / (ms[0] * 1e-3) / 1e12 / FP64_PEAK_TFS
                             if ms[0] else None,
                             "cholesky_frac": chol_flop / (ms[2] * 1e-3) / 1e12 / FP64_PEAK_TFS if ms[2] else None}})
    return out


def synthetic_section(seeds=(0, 1, 2)):
    """The paper's synthetic benchmark (Sec. V-D, Table III): X, Y ~ U(0,1),
    sigma = 0.1, M clipped at 0, n = 2000, m in {50, 100}, k in 3..6, solved to
    the paper's E(.;0) <= 1e-6.  The paper's MATLAB averages (CPU, 10 starts)
    are quoted as context."""
    import statistics
    import numpy as np
    import torch
    from paper_2101_08431_amd import NMF, default_options, synth
    table3 = {(50, 3): (3.31, 4.61662e2), (50, 4): (7.41, 4.56019e2), (50, 5): (6.98, 4.45449e2),
              (50, 6): (14.46, 4.36121e2), (100, 3): (4.05, 9.57337e2), (100, 4): (7.46, 9.54230e2),
              (100, 5): (11.77, 9.44857e2), (100, 6): (25.54, 9.35451e2)}
    rows = []
    for (m, k), (paper_s, paper_f) in table3.items():
        runs = []
        for seed in seeds:
            M, X0, Y0 = synth.make(dict(kind="uniform", n=2000, m=m, k=k, sigma=0.1), seed)
            ctx = NMF(M, k, X0, Y0, options=default_options(eps_tol=1e-6, max_ipm_iters=5000))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, rep = ctx.solve()
            torch.cuda.synchronize()
            runs.append({"seed": seed, "converged": st == 1, "ms": (time.perf_counter() - t0) * 1e3,
                         "E0": rep["E0"], "f": rep["f"], "ipm_iters": rep["ipm_iters"]})
            ctx.close()
        rows.append({"n": 2000, "m": m, "k": k, "runs": runs,
                     "median_ms": statistics.median(r["ms"] for r in runs),
                     "mean_f": statistics.mean(r["f"] for r in runs),
                     "paper_mean_cpu_s_matlab": paper_s, "paper_mean_f": paper_f,
                     "f_rel_to_paper": statistics.mean(r["f"] for r in runs) / paper_f - 1.0})
        log(f"synthetic m={m} k={k}: median {rows[-1]['median_ms']:.1f} ms, f {rows[-1]['mean_f']:.4e}")
    return {"workload": "uniform U(0,1), sigma 0.1 (Sec. V-D)", "eps_tol": 1e-6, "rows": rows}


def precision_section(steps):
    import numpy as np
    import oracle
    from paper_2101_08431_amd import synth
    M, X0, Y0 = synth.make("pdf_10000x2000_k10", 0)
    n, m = M.shape
    k = X0.shape[1]
    ref = oracle.anls(M, X0, Y0.T.copy(), exact_sweeps=5)
    scale = max(np.abs(ref["X"]).max(), np.abs(ref["Yt"]).max())
    f_ref = oracle.objective(M, ref["X"], ref["Yt"])
    res = {"workload": "pdf_10000x2000_k10", "n": n, "m": m, "k": k}
    for name, prec in (("fp64", 0), ("fp32", 1), ("bf16x2", 2)):
        ctx = make_ctx(M, X0, Y0, k, gram_precision=prec)
        ctx.anls_step(5, report=False)
        X, Y = ctx.factors()
        err = max(np.abs(X - ref["X"]).max(), np.abs(Y.T - ref["Yt"]).max()) / scale
        f = oracle.objective(M, X, Y.T.copy())
        ms, _, _ = time_graph_sweeps(ctx, steps, 5)
        ms4 = ctx.anls_profile(20)
        res[name] = {"ms_per_sweep": ms, "solves_per_s": (n + m) / (ms * 1e-3),
                     "stream_ms": [ms4[0], ms4[2]],
                     "stream_GBs": [(8 if prec == 0 else 4) * n * m / (t * 1e-3) / 1e9 for t in (ms4[0], ms4[2])],
                     "factor_rel_err_after_5_sweeps": err, "objective_rel_err": abs(f - f_ref) / f_ref}
        ctx.close()
    return res


def batching_section(count, sweeps):
    import numpy as np
    import torch
    from paper_2101_08431_amd import Batch, autotune, synth
    rng = np.random.default_rng(4)
    ctxs, solves = [], 0
    for p in range(count):
        n = int(rng.integers(500, 4001))
        m = int(rng.integers(100, 1001))
        k = int(rng.integers(2, 9))
        M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-3, sigma_relative=True), 10000 + p)
        ctxs.append(make_ctx(M, X0, Y0, k))
        solves += n + m
    torch.cuda.synchronize()
    # plain method: every problem's own four launches per sweep
    for c in ctxs:
        c.anls_step(1, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        for c in ctxs:
            c.anls_step(1, report=False)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / sweeps
    b = Batch(ctxs)
    waves, tuned_ms = autotune.tune_batch(b, sweeps=5, use_cache=False)
    b.step(sweeps, graph=True)
    b.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(sweeps, graph=True)
    e1.record(b.stream)
    b.sync()
    batch_ms = e0.elapsed_time(e1) / sweeps
    # the same batched sweeps launched eagerly (no graph)
    e0.record(b.stream)
    b.step(sweeps, graph=False)
    e1.record(b.stream)
    b.sync()
    eager_ms = e0.elapsed_time(e1) / sweeps
    b.close()
    return {"problems": count, "column_solves_per_sweep": solves,
            "plain_ms_per_sweep": plain_ms, "plain_solves_per_s": solves / (plain_ms * 1e-3),
            "batched_ms_per_sweep": batch_ms, "batched_solves_per_s": solves / (batch_ms * 1e-3),
            "batched_eager_ms_per_sweep": eager_ms,
            "speedup": plain_ms / batch_ms, "autotuned_waves": waves}


def grouping_section(ranks=(5, 10, 16), n=3000, m=500, warm=200, steps=50, cold=8):
    """Passive-set-grouped first solves (Sec. II grouping) against the
    per-problem loop: ms per sweep in the steady state (after `warm` sweeps,
    stable warm-start sets) and over the first `cold` sweeps from X0 = 0
    (sets churn)."""
    import numpy as np
    import torch
    from paper_2101_08431_amd import synth
    rows = []
    for k in ranks:
        M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-3, sigma_relative=True), 0)
        row = {"n": n, "m": m, "k": k}
        for grouped in (0, 1):
            tag = "grouped" if grouped else "per_problem"
            ctx = make_ctx(M, X0, Y0, k)
            ctx.set_nnls_grouping(grouped)
            row[f"{tag}_warm_ms_per_sweep"] = time_eager_sweeps(ctx, steps, warm)
            if grouped:
                xm, ym = ctx.masks()
                row["distinct_sets_x"] = int(np.unique(xm).size)
                row["distinct_sets_y"] = int(np.unique(ym).size)
            ctx.close()
            ctx = make_ctx(M, np.zeros_like(X0), Y0, k)
            ctx.set_nnls_grouping(grouped)
            torch.cuda.synchronize()
            row[f"{tag}_cold_ms_per_sweep"] = time_eager_sweeps(ctx, cold, 0)
            ctx.close()
        row["warm_speedup"] = row["per_problem_warm_ms_per_sweep"] / row["grouped_warm_ms_per_sweep"]
        row["cold_speedup"] = row["per_problem_cold_ms_per_sweep"] / row["grouped_cold_ms_per_sweep"]
        log(f"grouping k={k}: {row}")
        rows.append(row)
    return {"workload": f"pdf_{n}x{m}, ranks {list(ranks)}", "rows": rows}


def serving_section(seconds, rate=200.0, warm=1.0, plain=True):
    """64 streams (13 at n = 8000, k = 8, the rest n = 2000, k = 4), each
    starting at m = 64; Poisson arrivals at `rate`/s, each appending 16 columns
    to a uniformly chosen stream and re-solving stage 1 to the stop rule.  The
    same trace runs through the continuous-batching server and through the
    plain one-request-at-a-time method; latency counts from the scheduled
    arrival, requests arriving in the first `warm` s are not counted."""
    from paper_2101_08431_amd.serving import PlainServer, Request, Server, build_workload, summarize
    specs, reqs = build_workload(streams=64, rate=rate, seconds=seconds)
    log(f"serving: {len(reqs)} requests on 64 streams generated")
    res = {"streams": 64, "rate_per_s": rate, "seconds": seconds, "requests": len(reqs),
           "m_final_max": max(s.m_capacity for s in specs), "warmup_s": warm,
           "request": "append 16 columns, then warm-started stage-1 sweeps until the stop rule "
                      "(eps_STOL 1e-4) holds or 64 sweeps are done; E0_* give the KKT error E(.;0) of "
                      "eq. (10) each request ends at (stage-1 duals), the same in the served and plain runs"}
    for name, cls in (("served", Server), ("plain", PlainServer)) if plain else (("served", Server),):
        srv = cls(specs, sweeps_per_round=4, eps_stol=1e-4, request_sweeps=64, kkt=True)
        srv.open_all()
        log(f"serving: {name} streams open")
        t0 = time.perf_counter()
        rr = srv.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
        log(f"serving: {name} run done in {time.perf_counter() - t0:.1f} s")
        res[name] = summarize(rr, t_from=warm)
        res[name]["wall_s"] = time.perf_counter() - t0
        if name == "served":
            res[name]["rounds"] = srv.rounds
            res[name]["mean_batch"] = float(sum(srv.batch_sizes) / max(1, len(srv.batch_sizes)))
        srv.close_all()
    if plain:
        res["p99_speedup"] = res["plain"]["p99_ms"] / res["served"]["p99_ms"]
    return res


def cpu_baseline(M, X0, Y0, budget_s=15.0):
    import oracle
    n, m = M.shape
    t0 = time.perf_counter()
    oracle.anls(M, X0, Y0.T.copy(), exact_sweeps=2)
    per = (time.perf_counter() - t0) / 2
    sweeps = max(2, min(4000, int(budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    oracle.anls(M, X0, Y0.T.copy(), exact_sweeps=sweeps)
    dt = time.perf_counter() - t0
    return {"value": (n + m) * sweeps / dt, "unit": "solves/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{sweeps} ANLS sweeps of the same {n}x{m} k={X0.shape[1]} workload from the same start "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the full two-stage solves")
    ap.add_argument("--no-layers", action="store_true", help="skip the precision and batching sections")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="length of the serving arrival trace")
    ap.add_argument("--shape", default=None, metavar="XS,YS[,FX,FY]",
                    help="fix the stage-1 launch plan (x splits, y splits[, X-half one kernel, Y-half one "
                         "kernel: 1, 0 or -1 = automatic]) instead of autotuning it")
    ap.add_argument("--ipm-only", action="store_true",
                    help="only time stage-2 iterations on the headline workload (for profiling)")
    ap.add_argument("--batching-only", action="store_true",
                    help="only run the batching section (256 problems, for profiling)")
    ap.add_argument("--grouping-only", action="store_true",
                    help="only run the passive-set grouping section")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only run the mixed-precision interior-point section")
    ap.add_argument("--large-only", action="store_true",
                    help="only run the stage-2 section at 10000x2000x10")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 10 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 8, "copies": 10}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path in this library "
              "(the sharding design is written down, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2101_08431_amd import synth

    if args.ipm_only:
        print(json.dumps(ipm_section(args.workload)), flush=True)
        return
    if args.batching_only:
        print(json.dumps(batching_section(256, 20)), flush=True)
        return
    if args.grouping_only:
        print(json.dumps(grouping_section()), flush=True)
        return
    if args.mixed_only:
        print(json.dumps(mixed_section()), flush=True)
        return
    if args.large_only:
        print(json.dumps(ipm_large_section()), flush=True)
        return
    M, X0, Y0 = synth.make(args.workload, 0)
    n, m = M.shape
    k = X0.shape[1]
    ctx = make_ctx(M, X0, Y0, k)
    from paper_2101_08431_amd import autotune
    if args.shape:
        vals = [int(v) for v in args.shape.split(",")]
        ctx.set_launch_shape(vals[0], vals[1])
        if len(vals) == 4:
            ctx.set_launch_fusion(vals[2], vals[3])
        log(f"launch plan (x splits, y splits, X one kernel, Y one kernel) = {ctx.launch_plan()}, fixed")
    else:
        # the launch shapes whose HBM byte counters are on record (the
        # measured `traffic` of the roofline needs the shape that runs); in
        # wider sweeps the other shapes and the one-kernel halves did not win
        # at this size
        autotune.tune_single(ctx, use_cache=False, pairs=HEADLINE_SHAPES, try_fusion=False)
        log(f"autotuned launch plan (x splits, y splits, X one kernel, Y one kernel) = {ctx.launch_plan()}; "
            "fastest: " + ", ".join(f"{kk}: {v * 1e3:.1f} us" for kk, v in list(autotune.last_timings.items())[:6]))
    shape = ctx.launch_plan()
    ms_graph, wall_ms, ms_batch_eager = time_graph_sweeps(ctx, args.steps, args.warmup)
    ms_eager = time_eager_sweeps(ctx, args.steps, args.warmup)
    mode = "graph" if ms_graph <= ms_eager else "eager"
    ms_step = min(ms_graph, ms_eager)
    value = (n + m) / (ms_step * 1e-3)
    rl = roofline(ctx, n, m, k, shape, args.workload)
    _, rep = ctx.anls_step(0)
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "k": k,
                   "step": "one ANLS sweep (X stream + row NNLS, then Y stream + column NNLS, each half "
                           "two kernels or one), n + m NNLS solves",
                   "launch": mode, "graph_ms_per_step": ms_graph, "eager_ms_per_step": ms_eager,
                   "graph_wall_ms_timed": wall_ms, "batch_form_eager_ms_per_step": ms_batch_eager,
                   "launch_plan": {"x_splits": shape[0], "y_splits": shape[1], "x_one_kernel": shape[2],
                                   "y_one_kernel": shape[3]}},
        "roofline": rl,
        "nnls_solves_per_problem": rep["nnls_solves"] / max(1, rep["sweeps"] * (n + m)),
    }
    ctx.close()
    log(f"headline done: {ms_step * 1e3:.1f} us per sweep ({mode})")
    if not args.no_solve:
        log("stage-2 iteration timing")
        out["ipm_iteration"] = ipm_section(args.workload)
        out["roofline"]["stage2"] = out["ipm_iteration"]["roofline"]
        log("full solves")
        out["full_solve"] = full_solve(args.workload, list(range(10)), 1e-8, 5000)
        out["full_solve_1e-10"] = full_solve(args.workload, list(range(10)), 1e-10, 5000)
        log("stage 2 at 10000x2000x10")
        out["ipm_large"] = ipm_large_section()
        log("synthetic benchmark")
        out["synthetic"] = synthetic_section()
    if not args.no_layers:
        log("precision section")
        out["precision"] = precision_section(200)
        log("batching section")
        out["batching"] = batching_section(256, 10)
        out["grouping"] = grouping_section()
    if not args.no_serve:
        log("serving section")
        out["serving"] = serving_section(args.serve_seconds)
        # four times the arrival rate for a short trace: above what one request
        # at a time can serve
        out["serving_4x_load"] = serving_section(3.0, rate=800.0, warm=0.5)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(M, X0, Y0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
