"""Serving form on the GPU: continuous batching gives every request the result
it gets alone, and admission keeps open streams within the memory budget."""
import numpy as np
import pytest

from paper_2101_08431_amd import synth
from paper_2101_08431_amd.serving import PlainServer, Request, Server, StreamSpec, build_workload

pytestmark = pytest.mark.gpu


def small_workload(close_last=False):
    # 6 streams of two sizes, ~40 requests arriving faster than they finish
    return build_workload(streams=6, rate=300.0, seconds=0.15, m0=24, add=8, seed=3, big_every=3,
                          small=(300, 3), big=(700, 5), close_last=close_last)


def test_each_request_same_alone_and_in_the_mix():
    specs, reqs = small_workload()
    print(f"case serving mix vs alone: {len(reqs)} requests on 6 streams", flush=True)
    alone = PlainServer(specs, record=True, sweeps_per_round=4)
    alone.open_all()
    ra = alone.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
    alone.close_all()
    mix = Server(specs, record=True, sweeps_per_round=4, max_active=64)
    mix.open_all()
    rm = mix.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
    mix.close_all()
    assert max(mix.batch_sizes) > 1              # requests really shared the GPU
    for a, b in zip(ra, rm):
        assert a.rid == b.rid and a.sweeps == b.sweeps and a.sweeps > 0
        assert np.array_equal(a.result[0], b.result[0]) and np.array_equal(a.result[1], b.result[1])


def test_memory_admission_and_slots():
    specs, reqs = small_workload(close_last=True)
    from paper_2101_08431_amd import workspace_bytes
    from paper_2101_08431_amd.serving import _options
    sizes = sorted(workspace_bytes(s.n, s.m_capacity, s.k, _options(1e-6, 5000)) for s in specs)
    budget = sizes[-1] + sizes[-2]               # any two streams fit, never three
    print(f"case serving admission, budget {budget} bytes, 2 slots", flush=True)
    srv = Server(specs, record=True, hbm_budget=budget, max_active=2)
    out = srv.run(reqs)
    assert all(r.end is not None for r in out)
    assert srv.peak_in_use <= budget
    assert max(srv.batch_sizes) <= 2
    # the results are still the plain ones
    ref = PlainServer(specs, record=True)
    ra = ref.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
    for a, b in zip(ra, out):
        assert a.sweeps == b.sweeps and np.array_equal(a.result[1], b.result[1])


def test_mix_equals_alone_across_launch_shape_change():
    # streams that start small (one kernel per half) and grow past 2^18
    # entries (split kernels) while requests overlap: every request still ends
    # where it ends alone
    specs, reqs = build_workload(streams=5, rate=2000.0, seconds=0.02, m0=64, add=16, seed=5, big_every=5,
                                 small=(2000, 4), big=(2600, 5))
    print(f"case serving across shape change: {len(reqs)} requests on 5 streams", flush=True)
    alone = PlainServer(specs, record=True)
    alone.open_all()
    ra = alone.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
    alone.close_all()
    mix = Server(specs, record=True, max_active=64)
    mix.open_all()
    rm = mix.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
    mix.close_all()
    assert max(mix.batch_sizes) > 1
    for a, b in zip(ra, rm):
        assert a.rid == b.rid
        assert a.sweeps == b.sweeps, (a.rid, a.sid, a.sweeps, b.sweeps)
        assert np.array_equal(a.result[0], b.result[0]) and np.array_equal(a.result[1], b.result[1]), (a.rid, a.sid)
