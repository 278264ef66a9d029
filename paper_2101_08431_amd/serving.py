"""Serving form: resident streaming factorisations under continuous batching.

A *stream* is one growing factorisation in the streaming setting of Sec. II:
its M, X, Y and passive sets stay resident in the stream's device workspace.
A *request* appends new time columns to one stream; ``nmf_append_columns``
solves the new columns of Y warm-started from the neighbouring column, and
stage-1 sweeps (Alg. 1) then run until the stop rule of Sec. IV holds again
on the grown problem.  Requests of one stream run in arrival order.

``Server`` (continuous batching):
  * admission by HBM footprint: a stream's workspace is allocated only while
    the bytes of all open streams stay within ``hbm_budget``; otherwise it
    waits, first come first served, until a stream closes;
  * at most ``max_active`` requests are in flight;
  * the requests in flight share batched sweeps (``nmf_batch_*``; the batch is
    rebuilt on every join or leave with ``nmf_batch_create_static``, which
    allocates no device memory): rounds of
    ``sweeps_per_round`` sweeps, then a status poll; finished requests leave
    and waiting ones join between rounds, so new work enters while other
    requests are on the GPU;
  * a joining request's append runs on its stream's own HIP stream while the
    batch of the running requests executes.

A request ends when the stop rule of Sec. IV holds on the grown problem or
its sweep budget (``request_sweeps``) is spent, whichever comes first.

``PlainServer`` is the plain per-request method on the same kernels and the
same resident state: one request at a time in arrival order, each with its
own stage-1 sweeps (rounds of the same length).

A problem's sweeps inside a batch are bitwise the sweeps it would do alone and
its stop rule is evaluated on the device after every sweep, so each request's
result does not depend on what else is in flight.

Device work happens in the HIP library; this module only schedules it.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class StreamSpec:
    sid: int
    n: int
    k: int
    m_capacity: int
    M0: np.ndarray            # (n, m0) Fortran order
    X0: np.ndarray            # (n, k)
    Y0: np.ndarray            # (k, m0)


@dataclass
class Request:
    rid: int
    sid: int
    cols: np.ndarray          # (n, q) Fortran order
    arrival: float            # scheduled arrival, s after the run's start
    close: bool = False       # the stream closes after this request
    start: Optional[float] = None
    end: Optional[float] = None
    sweeps: int = 0
    solves: int = 0
    result: Optional[tuple] = None
    E0: Optional[float] = None   # E(.;0) of eq. (10) at the request's end point (stage-1 duals)

    @property
    def latency(self):
        return None if self.end is None else self.end - self.arrival


class _Stream:
    def __init__(self, spec: StreamSpec):
        self.spec = spec
        self.ctx = None
        self.hip_stream = None
        self.queue = collections.deque()
        self.active: Optional[Request] = None
        self.sweeps = 0           # cumulative stage-1 sweeps of the context
        self.nbytes = 0
        self.closed = False


def _options(eps_stol, max_sweeps):
    from ._lib import default_options
    return default_options(eps_stol=eps_stol, max_anls_sweeps=max_sweeps, with_ipm=0)


class _Base:
    """eps_stol: the stop rule of every solve; initial_sweeps: sweep budget of
    the solve of a stream's first window; request_sweeps: sweep budget of each
    request (a request ends when the stop rule holds or its budget is spent);
    sweeps_per_round: sweeps between two status checks."""

    def __init__(self, specs: List[StreamSpec], eps_stol=1e-4, initial_sweeps=2000, request_sweeps=64,
                 sweeps_per_round=4, hbm_budget=None, record=False, kkt=False):
        import torch
        from ._lib import workspace_bytes
        self.torch = torch
        self.streams = {s.sid: _Stream(s) for s in specs}
        self.opts = _options(eps_stol, initial_sweeps)
        self.request_sweeps = int(request_sweeps)
        self.T = int(sweeps_per_round)
        self.record = record
        self.kkt = bool(kkt)   # measure E(.;0) of every finished request (after its end time)
        for st in self.streams.values():
            st.nbytes = workspace_bytes(st.spec.n, st.spec.m_capacity, st.spec.k, self.opts)
        total = sum(st.nbytes for st in self.streams.values())
        self.budget = total if hbm_budget is None else int(hbm_budget)
        self.in_use = 0
        self.peak_in_use = 0
        self.wait_open = collections.deque()
        self.t0 = None

    # -- streams
    def _can_open(self, st):
        return self.in_use + st.nbytes <= self.budget

    def _create(self, st):
        from ._lib import NMF
        st.hip_stream = self.torch.cuda.Stream()
        sp = st.spec
        st.ctx = NMF(sp.M0, sp.k, sp.X0, sp.Y0, m_capacity=sp.m_capacity, options=self.opts,
                     stream=st.hip_stream)
        self.in_use += st.nbytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)

    def _open(self, st):
        """Allocate the stream's workspace and solve its first window (Alg. 1
        from the given start until the stop rule holds or the initial budget
        is spent), then set the per-request budget."""
        self._create(st)
        while True:
            code, rep = st.ctx.anls_step(64)
            if code == 1:
                break
        st.sweeps = rep["sweeps"]
        st.ctx.set_anls_budget(self.request_sweeps)

    def open_all(self):
        """Open every stream that fits the budget (before a timed run).  The
        first windows are solved together in batched sweeps; each ends where
        its own solve would."""
        from ._lib import Batch
        new = []
        for st in self.streams.values():
            if st.ctx is None and not st.closed and self._can_open(st):
                self._create(st)
                new.append(st)
        if not new:
            return
        self.torch.cuda.synchronize()
        b = Batch([st.ctx for st in new])
        while True:
            b.step(32, graph=False)
            conv, sweeps = b.poll()
            if conv.all():
                break
        b.close()
        for st, sw in zip(new, sweeps):
            st.sweeps = int(sw)
            st.ctx.set_anls_budget(self.request_sweeps)

    def close_all(self):
        for st in self.streams.values():
            if st.ctx is not None:
                self._close(st)

    def _close(self, st):
        st.ctx.close()
        st.ctx = None
        st.closed = True
        self.in_use -= st.nbytes

    def _now(self):
        return time.perf_counter() - self.t0

    def _finish(self, st, req, sweeps_total):
        req.end = self._now()
        req.sweeps = int(sweeps_total - st.sweeps)
        st.sweeps = int(sweeps_total)
        m = st.ctx.m
        req.solves = req.sweeps * (st.spec.n + m) + m
        if self.record:
            req.result = st.ctx.factors()
        if self.kkt:
            req.E0 = float(st.ctx.report()["E0"])
        st.active = None
        if req.close:
            self._close(st)


class PlainServer(_Base):
    """One request at a time, in arrival order."""

    def run(self, requests: List[Request]):
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        for req in reqs:
            now = self._now()
            if now < req.arrival:
                time.sleep(req.arrival - now)
            st = self.streams[req.sid]
            if st.ctx is None:
                if st.closed or not self._can_open(st):
                    raise RuntimeError(f"stream {req.sid} cannot be opened")
                self._open(st)
            req.start = self._now()
            st.active = req
            st.ctx.append_columns(req.cols)
            while True:
                code, rep = st.ctx.anls_step(self.T)
                if code == 1:
                    break
            self._finish(st, req, rep["sweeps"])
        return reqs


class Server(_Base):
    """Continuous batching of stage-1 sweeps over the requests in flight."""

    def __init__(self, specs, max_active=64, use_graph=False, **kw):
        super().__init__(specs, **kw)
        self.max_active = int(max_active)
        self.use_graph = bool(use_graph)
        self.rounds = 0
        self.batch_sizes = []

    def _admit_streams(self):
        while self.wait_open:
            st = self.wait_open[0]
            if not self._can_open(st):
                break
            self.wait_open.popleft()
            self._open(st)

    def run(self, requests: List[Request]):
        from ._lib import Batch
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        ready = collections.deque()    # streams with a queued request, in arrival order
        running: List[_Stream] = []    # streams whose request is in the batch
        joined: List[_Stream] = []     # appended, join at the next round
        batch = None
        batch_members: List[_Stream] = []
        dirty = False
        self.t0 = time.perf_counter()
        remaining = len(pending)
        while remaining > 0:
            now = self._now()
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                st = self.streams[req.sid]
                st.queue.append(req)
                if st.ctx is None and not st.closed and st not in self.wait_open:
                    self.wait_open.append(st)
                if st.active is None and st not in ready:
                    ready.append(st)
            self._admit_streams()
            # membership for this round: a batch holds each problem's shape as
            # it was when the batch was built, so any join or leave rebuilds it
            if joined:
                running.extend(joined)
                joined = []
                dirty = True
            if running and dirty:
                if batch is not None:
                    batch.close()
                # the batch tables live in the library's own per-device array
                # (nmf_batch_create_static): a rebuild allocates nothing and
                # waits only for the member streams
                batch = Batch([s.ctx for s in running], stream=self._batch_stream(), static=True)
                batch_members = list(running)
                dirty = False
            if running:
                batch.step(self.T, graph=self.use_graph)
                self.rounds += 1
                self.batch_sizes.append(len(running))
            # requests join while the batch runs: their appends go on their own streams
            n_active = len(running)
            skipped = collections.deque()
            while ready and n_active < self.max_active:
                st = ready.popleft()
                if not st.queue:
                    continue
                if st.ctx is None:          # waiting for memory
                    skipped.append(st)
                    continue
                req = st.queue.popleft()
                req.start = self._now()
                st.active = req
                st.ctx.append_columns(req.cols)
                joined.append(st)
                n_active += 1
            skipped.extend(ready)
            ready = skipped
            if running:
                conv, sweeps = batch.poll()
                still = []
                for st, c, sw in zip(batch_members, conv, sweeps):
                    if c:
                        req = st.active
                        self._finish(st, req, sw)
                        remaining -= 1
                        if st.queue and st.ctx is not None and st not in ready:
                            ready.append(st)
                    else:
                        still.append(st)
                if len(still) != len(running):
                    dirty = True
                running = still
            elif not joined:
                # idle: wait for the next arrival (or for memory that never frees)
                if pending:
                    wait = pending[0].arrival - self._now()
                    if wait > 0:
                        time.sleep(wait)
                elif not ready or all(s.ctx is None for s in ready):
                    raise RuntimeError("requests left that can never be admitted")
        if batch is not None:
            batch.close()
        torch.cuda.synchronize()
        return sorted(requests, key=lambda r: r.arrival)

    def _batch_stream(self):
        if not hasattr(self, "_bs"):
            self._bs = self.torch.cuda.Stream()
        return self._bs


def summarize(reqs: List[Request], t_from=0.0, t_to=None):
    """Latency percentiles (ms) and throughput over requests that arrived in
    [t_from, t_to)."""
    sel = [r for r in reqs if r.arrival >= t_from and (t_to is None or r.arrival < t_to) and r.end is not None]
    if not sel:
        return {"requests": 0}
    lat = np.array([r.latency for r in sel]) * 1e3
    span = max(r.end for r in sel) - min(r.arrival for r in sel)
    solves = sum(r.solves for r in sel)
    out = {"requests": len(sel), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
           "sweeps_per_request": float(np.mean([r.sweeps for r in sel])),
           "requests_per_s": len(sel) / span if span > 0 else None,
           "solves_per_s": solves / span if span > 0 else None}
    E = [r.E0 for r in sel if r.E0 is not None]
    if E:
        out["E0_median"] = float(np.median(E))
        out["E0_p99"] = float(np.percentile(E, 99))
        out["E0_max"] = float(np.max(E))
    return out


def build_workload(streams=64, rate=200.0, seconds=20.0, m0=64, add=16, seed=7, big_every=5,
                   small=(2000, 4), big=(8000, 8), close_last=False):
    """Stream specs and the request list of the serving workload: ``streams``
    streams (every ``big_every``-th of size ``big``, the rest ``small``), each
    starting with ``m0`` columns; Poisson arrivals at ``rate``/s in total for
    ``seconds``, each request appending ``add`` columns to a uniformly chosen
    stream."""
    from . import synth
    sizes = synth.serving_streams(streams, big_every, small, big)
    trace = synth.serving_trace(streams, rate, seconds, seed)
    per = collections.Counter(s for _, s in trace)
    specs, blocks = [], {}
    for s, (n, k) in enumerate(sizes):
        cnt = per.get(s, 0)
        M0, bl, X0, Y0 = synth.serving_stream_data(n, k, m0, add, cnt, seed=20000 + 97 * seed + s)
        specs.append(StreamSpec(s, n, k, m0 + add * cnt, M0, X0, Y0))
        blocks[s] = bl
    reqs, used = [], collections.Counter()
    last = {s: max(q for q, (_, ss) in enumerate(trace) if ss == s) for s in per}
    for q, (t, s) in enumerate(trace):
        reqs.append(Request(q, s, blocks[s][used[s]], t, close=close_last and last[s] == q))
        used[s] += 1
    return specs, reqs
