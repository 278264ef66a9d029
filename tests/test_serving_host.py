"""Host-side pieces of the serving form: the seeded request trace, the stream
data and the latency summary (no GPU needed)."""
import numpy as np
import pytest

from paper_2101_08431_amd import synth
from paper_2101_08431_amd.serving import Request, summarize


def test_trace_is_poisson_at_the_given_rate():
    tr = synth.serving_trace(64, 200.0, 50.0, seed=7)
    t = np.array([a for a, _ in tr])
    assert np.all(np.diff(t) > 0) and t[-1] < 50.0
    assert len(tr) == pytest.approx(200.0 * 50.0, rel=0.05)
    gaps = np.diff(t)
    assert gaps.mean() == pytest.approx(1 / 200.0, rel=0.05)
    assert gaps.std() == pytest.approx(gaps.mean(), rel=0.08)   # exponential: sd = mean
    streams = np.bincount([s for _, s in tr], minlength=64)
    assert streams.min() > 0.6 * streams.mean() and streams.max() < 1.4 * streams.mean()
    assert synth.serving_trace(64, 200.0, 50.0, seed=7) == tr


def test_stream_sizes():
    sz = synth.serving_streams(64)
    assert sz.count((8000, 8)) == 13 and sz.count((2000, 4)) == 51
    assert all(sz[s] == (8000, 8) for s in range(0, 64, 5))


def test_stream_blocks_extend_the_first_window():
    M0, blocks, X0, Y0 = synth.serving_stream_data(50, 3, 8, 4, 3, seed=11)
    full, _, _ = synth.pdf_like(50, 20, 3, 11, sigma=1e-3, sigma_relative=True, m_horizon=20)
    joined = np.hstack([M0] + blocks)
    assert np.array_equal(joined, full)
    assert all(b.flags["F_CONTIGUOUS"] and b.shape == (50, 4) for b in blocks)
    assert X0.shape == (50, 3) and Y0.shape == (3, 8) and (X0 >= 0).all() and (Y0 >= 0).all()


def test_summary_percentiles():
    reqs = []
    for q in range(100):
        r = Request(q, 0, None, arrival=0.01 * q)
        r.end = r.arrival + 0.001 * (q + 1)
        r.sweeps, r.solves = 2, 10
        reqs.append(r)
    s = summarize(reqs)
    assert s["requests"] == 100
    assert s["p50_ms"] == pytest.approx(np.percentile(np.arange(1, 101), 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(np.arange(1, 101), 99))
    assert s["max_ms"] == pytest.approx(100.0)
    assert summarize(reqs, t_from=0.5)["requests"] == 50
