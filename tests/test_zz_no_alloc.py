"""nmf_batch_create_static (no device allocation; the batch tables live in the
library's own per-device array) against nmf_batch_create with a caller
workspace: the same contexts swept through either batch end bitwise equal, and
equal to the FP64 oracle's sweeps.  Two static batches in a row, the second
over fewer and smaller problems, so the second call reuses the array that the
first filled."""
import ctypes

import numpy as np
import pytest

from paper_2101_08431_amd import synth

pytestmark = pytest.mark.gpu

SWEEPS = 6


def problems(count, seed0, nmax, mmax):
    rng = np.random.default_rng(seed0)
    out = []
    for q in range(count):
        n = int(rng.integers(80, nmax))
        m = int(rng.integers(16, mmax))
        k = int(rng.integers(2, 9))
        M, X0, Y0 = synth.make(dict(kind="pdf", n=n, m=m, k=k, sigma=1e-3, sigma_relative=True), seed0 + q)
        out.append((M, X0, Y0, k))
    return out


def contexts(probs):
    from paper_2101_08431_amd import NMF, default_options
    opts = dict(eps_stol=-1.0, max_anls_sweeps=1 << 30, with_ipm=0)
    return [NMF(M, k, X0, Y0, options=default_options(**opts)) for (M, X0, Y0, k) in probs]


def run(probs, static):
    import torch
    from paper_2101_08431_amd import Batch
    ctxs = contexts(probs)
    b = Batch(ctxs, static=static)
    b.step(SWEEPS, graph=False)
    conv, sweeps = b.poll()
    assert (sweeps == SWEEPS).all(), sweeps
    b.close()
    torch.cuda.synchronize()
    out = [c.factors() for c in ctxs]
    for c in ctxs:
        c.close()
    return out


@pytest.mark.parametrize("call", [0, 1])
def test_static_batch_matches_workspace_batch_and_oracle(call, orc):
    # call 0: 9 problems up to 1500 x 300; call 1: 4 problems up to 400 x 60
    count, seed0, nmax, mmax = [(9, 31000, 1500, 300), (4, 31100, 400, 60)][call]
    probs = problems(count, seed0, nmax, mmax)
    print(f"case static batch call {call}: {count} problems, n < {nmax}, m < {mmax}", flush=True)
    ref = run(probs, static=False)
    got = run(probs, static=True)
    for (M, X0, Y0, k), (X, Y), (Xs, Ys) in zip(probs, ref, got):
        assert np.array_equal(Xs, X) and np.array_equal(Ys, Y)
        o = orc.anls(M, X0, Y0.T.copy(), exact_sweeps=SWEEPS)
        scale = max(np.abs(o["X"]).max(), np.abs(o["Yt"]).max())
        err = max(np.abs(Xs - o["X"]).max(), np.abs(Ys.T - o["Yt"]).max()) / scale
        assert err <= 1e-8, err


def test_static_batch_rejects_oversized_count():
    import torch
    from paper_2101_08431_amd import _lib
    L = _lib.load()
    n = _lib.BATCH_STATIC_MAX + 1
    arr = (ctypes.c_void_p * n)()
    out = ctypes.c_void_p()
    s = torch.cuda.current_stream()
    st = L.nmf_batch_create_static(arr, n, ctypes.c_void_p(s.cuda_stream), ctypes.byref(out))
    assert st == _lib.NMF_ECAPACITY
    assert b"static batch limit" in L.nmf_last_error(None)
