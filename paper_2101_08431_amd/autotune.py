"""Launch-shape autotuner for the stage-1 kernels.

The shape knobs are the column splits of the X-half streaming kernel and the
row splits of the Y-half one (more splits: more waves streaming M, more
partial sums to reduce).  The tuner times candidate shapes on the device with
the library's own per-kernel event profiler (single problem) or with replayed
batched sweeps (batch), keeps the fastest, and caches the choice in a JSON file
(``NMF_TUNE_CACHE``, default ``~/.cache/nmf_mi355x_tune.json``) keyed by the
problem signature.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

XTILE, SWAVES, STHR = 64, 8, 512
last_timings = {}   # ms per sweep of every shape the last tune_single call timed


def _cache_path():
    return os.environ.get("NMF_TUNE_CACHE", os.path.expanduser("~/.cache/nmf_mi355x_tune.json"))


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def splits_for_waves(n, m, k, waves):
    """Split counts that give about `waves` streaming waves per kernel.  A
    single split (one kernel per half) is kept for matrices of at most 2^18
    entries, as the library's automatic shape does; larger ones keep at least
    two splits, so their NNLS runs in its own kernel."""
    lo = 1 if n * m <= (1 << 18) else 2
    tn = math.ceil(n / XTILE)
    xs = max(lo, min(math.ceil(waves / (SWAVES * tn)), 64, m))
    j = max(1, 64 // k)
    tm = math.ceil(m / j)
    ys = max(lo, min(math.ceil(waves / (SWAVES * tm)), max(1, n // STHR), 64, n))
    return min(xs, m), min(ys, n)


FUSE_KMAX = 7   # above this rank the one-kernel halves spill registers


def _apply_single(ctx, xs, ys, fx, fy):
    ctx.set_launch_shape(xs, ys)
    ctx.set_launch_fusion(fx, fy)


def tune_single(ctx, xs_cands=(1, 2, 4, 8, 11, 16), ys_cands=(1, 2, 3, 4, 6), sweeps=30, use_cache=True,
                pairs=None, try_fusion=True):
    """Pick the stage-1 launch plan of one context, (x_splits, y_splits,
    fuse_x, fuse_y), by timing back-to-back sweeps of each candidate: every
    split pair with the automatic kernel split (one kernel per half exactly at
    a single split) and, for ranks up to FUSE_KMAX, with each half forced into
    one kernel.  `pairs` (a list of (x_splits, y_splits)) replaces the product
    of the two candidate lists; try_fusion=False keeps the automatic kernel
    split only.  Returns the choice and sets it.  The sweeps advance the
    factorisation, so tune a context whose stop rule cannot hold yet (or a
    copy of one)."""
    shapes = list(pairs) if pairs is not None else [(xs, ys) for xs in xs_cands for ys in ys_cands]
    key = (f"single2:{ctx.n}:{ctx.m}:{ctx.k}:{int(ctx.options.gram_precision)}:"
           + hashlib.sha1(json.dumps([shapes, try_fusion]).encode()).hexdigest()[:8])
    cache = _load() if use_cache else {}
    if key in cache:
        choice = tuple(cache[key]["choice"])
        _apply_single(ctx, *choice)
        return choice
    import torch
    fusions = [(-1, -1)] + ([(1, -1), (-1, 1), (1, 1)] if try_fusion and ctx.k <= FUSE_KMAX else [])
    timings = {}
    for xs, ys in shapes:
        for fx, fy in fusions:
            _apply_single(ctx, xs, ys, fx, fy)
            plan = ctx.launch_plan()
            if any(plan == ctx_plan for ctx_plan, _ in timings.values()):
                continue   # the same launch plan as an earlier candidate
            ctx.anls_step(3, report=False)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            ctx.anls_step(sweeps, report=False)
            e1.record(ctx.stream)
            e1.synchronize()
            timings[(xs, ys, fx, fy)] = (plan, e0.elapsed_time(e1) / sweeps)
    best = min(timings, key=lambda c: timings[c][1])
    _apply_single(ctx, *best)
    global last_timings
    last_timings = {_label(timings[c][0]): timings[c][1] for c in sorted(timings, key=lambda c: timings[c][1])}
    cache = _load()
    cache[key] = {"choice": list(best), "ms": timings[best][1],
                  "tried": {_label(p): t for p, t in timings.values()}}
    _store(cache)
    return best


def _label(plan):
    """'xs,ys' plus the halves that run as one kernel, e.g. '8,3 fused x'."""
    xs, ys, fx, fy = plan
    tag = {(False, False): "", (True, False): " fused x", (False, True): " fused y", (True, True): " fused x,y"}
    return f"{xs},{ys}{tag[(fx, fy)]}"


def tune_batch(batch, waves_cands=(256, 512, 1024, 2048, 4096), sweeps=10, use_cache=True):
    """Pick one target wave count for every problem of a batch by timing replayed
    batched sweeps; sets the shapes and returns (waves, ms_per_sweep)."""
    import torch
    sig = hashlib.sha1(json.dumps([(c.n, c.m, c.k, int(c.options.gram_precision))
                                   for c in batch.contexts]).encode()).hexdigest()[:16]
    key = f"batch:{len(batch.contexts)}:{sig}"
    cache = _load() if use_cache else {}

    def apply(w):
        for c in batch.contexts:
            c.set_launch_shape(*splits_for_waves(c.n, c.m, c.k, w))
        batch.refresh()

    if key in cache:
        apply(cache[key]["choice"])
        return cache[key]["choice"], cache[key]["ms"]
    timings = {}
    for w in waves_cands:
        apply(w)
        batch.step(sweeps, graph=True)
        batch.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(batch.stream)
        batch.step(sweeps, graph=True)
        e1.record(batch.stream)
        batch.sync()
        timings[w] = e0.elapsed_time(e1) / sweeps
    best = min(timings, key=timings.get)
    apply(best)
    cache = _load()
    cache[key] = {"choice": best, "ms": timings[best], "tried": {str(k): v for k, v in timings.items()},
                  "when": time.time()}
    _store(cache)
    return best, timings[best]
