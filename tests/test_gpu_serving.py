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


def test_served_requests_match_oracle(orc):
    # fixed sweep budgets (no stop rule) make every request's work a known
    # count, so the oracle can replay each stream: its first window for
    # `initial` sweeps, then per request the Y-half over all columns with the
    # appended ones (nmf_append_columns) and `per_req` sweeps (Alg. 1)
    initial, per_req = 30, 6
    specs, reqs = build_workload(streams=4, rate=400.0, seconds=0.03, m0=24, add=8, seed=11, big_every=2,
                                 small=(300, 3), big=(600, 5))
    print(f"case served requests vs oracle: {len(reqs)} requests on 4 streams", flush=True)
    srv = Server(specs, eps_stol=-1.0, initial_sweeps=initial, request_sweeps=per_req, record=True,
                 sweeps_per_round=3, max_active=64)
    srv.open_all()
    out = srv.run([Request(r.rid, r.sid, r.cols, r.arrival) for r in reqs])
    srv.close_all()
    assert max(srv.batch_sizes) > 1
    state = {}
    for sp in specs:
        ref = orc.anls(sp.M0, sp.X0, sp.Y0.T.copy(), exact_sweeps=initial)
        state[sp.sid] = (np.asfortranarray(sp.M0), ref["X"], ref["Yt"])
    for r in out:   # arrival order is each stream's request order
        M, X, Yt = state[r.sid]
        M = np.asfortranarray(np.hstack([M, r.cols]))
        Yt = np.vstack([Yt, np.zeros((r.cols.shape[1], Yt.shape[1]))])
        Yt, _, bad = orc.half_y(M, X, Yt)
        assert bad == 0
        ref = orc.anls(M, X, Yt, exact_sweeps=per_req)
        state[r.sid] = (M, ref["X"], ref["Yt"])
        assert r.sweeps == per_req
        Xg, Yg = r.result
        scale = max(np.abs(ref["X"]).max(), np.abs(ref["Yt"]).max())
        err = max(np.abs(Xg - ref["X"]).max(), np.abs(Yg.T - ref["Yt"]).max()) / scale
        assert err <= 1e-8, (r.rid, r.sid, err)
