"""Serving form: a continuous-batching request loop over the c4m stepper.

Requests (cavity simulations of different sizes and step counts) arrive over
time.  Work is issued in units that run asynchronously on the device:
  * a cohort per dimension: every active request of that dimension, stepped
    together as one batch (2D: persistent launches; 3D: every launch of the
    step over all members), re-formed only when its membership changed and
    no chunk of it is in flight;
  * with a backend that does not batch a dimension, each such request on
    its own side stream.
A unit advances by a chunk of k = min(chunk, fewest remaining steps among
its members) steps, so nobody overshoots, and records a completion event.
The loop polls those events: a finished chunk retires the requests it
completed (fields copied out, memory released) and the unit is relaunched at
once; arrivals are queued and admitted in arrival order while their device
footprint fits the HBM budget and the active count is below max_active (a
request that does not fit waits; up to max_skip smaller later ones may pass
it); at most admit_per_poll requests are created per pass of the loop, so
polling and relaunching keep going while a burst of arrivals is admitted.
Nothing waits for the whole device.  The device backend sets a request up
(workspace, initial fields, the step graphs of its chunk lengths) on a
worker thread and a private stream, then hands it to its compute stream, so
set-up never waits behind other requests' queued chunks; the request joins
its unit when that is done.  Latency of a request is
completion minus arrival; the loop reports p50/p99 latency and completed
cell-steps per second.  Fields stay resident from admission to retirement.

The backend is pluggable so the scheduling logic is testable on the CPU
(tests/test_serve_cpu.py); DeviceBackend drives libc4m.so.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    id: int
    t_arrive: float
    dim: int
    n: int
    k: tuple
    steps: int
    amp: float = 1.0
    r: float = 0.5
    t_admit: float = -1.0
    t_done: float = -1.0
    remaining: int = 0
    handle: object = None
    result: dict = None
    side: int = 0

    @property
    def cells(self) -> int:
        return self.n ** self.dim


class DeviceBackend:
    """Requests on the GPU through libc4m.so (PyTorch for memory and
    streams); completion of a chunk is an event recorded on its stream."""

    def __init__(self, n_side_streams: int = 4, settings: dict | None = None, keep_results: bool = False,
                 chunk: int = 96, workers: int = 2, per_stream: int = 2, batch_3d: bool = True):
        import torch
        from .problem import make_config, workspace_bytes
        self.torch = torch
        self._make_config = make_config
        self._workspace_bytes = workspace_bytes
        self.settings = dict(settings or {})
        self.main = torch.cuda.Stream()
        self.side = [torch.cuda.Stream() for _ in range(n_side_streams)]
        self.keep_results = keep_results
        self._batch = {}                # dim -> batch of the cohort
        self._members = {}              # dim -> member handles of that batch
        self.cohort_dims = (2, 3) if batch_3d else (2,)
        self.main3 = torch.cuda.Stream()
        self._next_side = 0
        self.chunk = int(chunk)
        self.per_stream = int(per_stream)
        self._inflight = {}             # side stream index -> chunks in flight
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=workers)
        self._local = threading.local()
        self._lock = threading.Lock()
        self.host_s = {"create": 0.0, "launch_2d": 0.0, "reform_2d": 0.0, "launch_3d": 0.0, "finish": 0.0}
        self.reforms = 0

    def footprint(self, req: Request) -> int:
        return self._workspace_bytes(self._make_config(req.dim, req.n, req.r, **self.settings))

    def create(self, req: Request):
        """Starts the set-up of a request; returns a future of its handle."""
        if req.dim == 2:
            stream = self.main
        elif 3 in self.cohort_dims:
            stream = self.main3
        else:
            req.side = self._next_side % len(self.side)
            stream = self.side[req.side]
            self._next_side += 1
        return self._pool.submit(self._create, req, stream)

    def can_launch(self, req: Request) -> bool:
        """A 3D request launches only while its stream has fewer than
        per_stream chunks queued: every step is some fifty kernels, and a
        deep backlog would block the loop in the launch."""
        return req.dim in self.cohort_dims or self._inflight.get(req.side, 0) < self.per_stream

    def _create(self, req: Request, stream):
        from workloads import mode_fields
        from .problem import Problem
        t = time.perf_counter()
        setup = getattr(self._local, "stream", None)
        if setup is None:
            setup = self._local.stream = self.torch.cuda.Stream()
        kw = dict(self.settings)
        if req.dim == 3 and 3 in self.cohort_dims:
            # a 3D cohort changes often: its steps are launched directly
            from ._lib import FLAG_DIRECT
            kw["flags"] = kw.get("flags", 0) | FLAG_DIRECT
        p = Problem(req.dim, req.n, req.r, stream=setup, **kw)
        t1 = time.perf_counter()
        h = 1.0 / req.n
        init = mode_fields(req.dim, req.n, req.k, 0.0, req.r * h / 2, amp=req.amp)
        t2 = time.perf_counter()
        for name in p.fields():
            p.set(name, init[name])
        t3 = time.perf_counter()
        if req.dim == 3 and 3 not in self.cohort_dims:     # the graphs of its chunk lengths
            p.prepare(min(self.chunk, req.steps))
            if req.steps % self.chunk:
                p.prepare(req.steps % self.chunk)
        t4 = time.perf_counter()
        p.set_stream(stream)
        t5 = time.perf_counter()
        with self._lock:
            for key, dt in (("create", t5 - t), ("c_problem", t1 - t), ("c_fields_host", t2 - t1),
                            ("c_set", t3 - t2), ("c_prepare", t4 - t3), ("c_set_stream", t5 - t4)):
                self.host_s[key] = self.host_s.get(key, 0.0) + dt
        return p

    def launch(self, reqs, k: int):
        """Start k steps of a unit (the 2D cohort or one 3D request);
        returns the event that marks its end."""
        from .batch import Batch
        t = time.perf_counter()
        dim = reqs[0].dim
        if dim in self.cohort_dims:
            stream = self.main if dim == 2 else self.main3
            key = tuple(id(r.handle) for r in reqs)
            if key != self._members.get(dim):
                if self._batch.get(dim) is not None:
                    self._batch[dim].close()
                self._batch[dim] = Batch.from_problems([r.handle for r in reqs], stream=stream)
                self._members[dim] = key
                self.reforms += 1
                t1 = time.perf_counter()
                self.host_s["reform_%dd" % dim] = self.host_s.get("reform_%dd" % dim, 0.0) + t1 - t
                t = t1
            self._batch[dim].step(k)
            self.host_s["launch_%dd" % dim] = self.host_s.get("launch_%dd" % dim, 0.0) + time.perf_counter() - t
        else:
            reqs[0].handle.step(k)
            stream = reqs[0].handle.stream
            self._inflight[reqs[0].side] = self._inflight.get(reqs[0].side, 0) + 1
            self.host_s["launch_3d"] += time.perf_counter() - t
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return (ev, None if dim in self.cohort_dims else reqs[0].side)

    def done(self, token) -> bool:
        ev, side = token
        if not ev.query():
            return False
        if side is not None:
            self._inflight[side] -= 1
        return True

    def idle(self):
        time.sleep(2e-4)

    def finish(self, req: Request):
        t = time.perf_counter()
        self._finish(req, self.keep_results)
        self.host_s["finish"] += time.perf_counter() - t

    def drain(self):
        self.torch.cuda.synchronize()
        self._inflight.clear()

    def abandon(self, req: Request):
        self._finish(req, False)

    def _finish(self, req: Request, keep: bool):
        names = ["ez", "hx", "hy"] if req.dim == 2 else ["ex", "ey", "ez", "hx", "hy", "hz"]
        if keep:
            req.result = {a: req.handle.get(a) for a in names}
        b = self._batch.get(req.dim)
        if b is not None and id(req.handle) in self._members.get(req.dim, ()):
            b.close()                           # the batch references this problem
            self._batch[req.dim] = None
            self._members[req.dim] = ()
        req.handle.close()
        req.handle = None

    def close(self):
        self._pool.shutdown(wait=True)
        for dim, b in self._batch.items():
            if b is not None:
                b.close()
        self._batch = {}
        self._members = {}


class Server:
    def __init__(self, backend, hbm_budget: int, chunk: int = 50, max_active: int = 32, max_skip: int = 8,
                 admit_per_poll: int = 4, clock=time.perf_counter, chunk_3d: int | None = None):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.max_active = int(max_active)
        self.max_skip = int(max_skip)
        self.admit_per_poll = int(admit_per_poll)
        self.chunk_3d = int(chunk_3d) if chunk_3d else self.chunk
        self.clock = clock
        self.in_use = 0
        self.peak_in_use = 0

    def run(self, requests, time_limit: float | None = None, progress=None, progress_every: float = 20.0) -> dict:
        """Serve `requests`; `progress(text)` (if given) is called about every
        `progress_every` seconds with the counts so far."""
        pending = sorted(requests, key=lambda q: q.t_arrive)
        queue, done = [], []
        active2, active3 = [], []
        starting = []               # admitted, set-up still running (backend futures)
        flight = {}                 # unit key -> (token, members, k); -dim: a cohort, request id + 1: one request
        footprint = {}
        t0 = self.clock()
        i = 0
        chunks = 0
        executed = 0.0              # cell-steps of finished chunks, finished requests or not
        next_report = progress_every
        while i < len(pending) or queue or active2 or active3 or starting:
            now = self.clock() - t0
            if progress is not None and now >= next_report:
                next_report += progress_every
                progress(f"t={now:.0f}s arrived={i} queued={len(queue)} active={len(active2) + len(active3)} "
                         f"done={len(done)} executed={executed / max(now, 1e-9) / 1e6:.0f} Mcell-steps/s")
            if time_limit is not None and now > time_limit:
                break
            while i < len(pending) and pending[i].t_arrive <= now:
                queue.append(pending[i])
                i += 1
            progressed = False
            # finished chunks: retire the requests they completed
            for key in list(flight):
                token, members, k = flight[key]
                if not self.backend.done(token):
                    continue
                del flight[key]
                progressed = True
                t_end = self.clock() - t0
                for r in members:
                    executed += float(r.cells) * k
                    r.remaining -= k
                    if r.remaining <= 0:
                        r.t_done = t_end
                        self.backend.finish(r)
                        self.in_use -= footprint[r.id]
                        done.append(r)
                        (active2 if r.dim == 2 else active3).remove(r)
            # requests whose set-up finished join their unit
            for q in list(starting):
                if q.handle.done():
                    q.handle = q.handle.result()
                    starting.remove(q)
                    (active2 if q.dim == 2 else active3).append(q)
                    progressed = True
            # admission by footprint, arrival order with bounded skipping
            skipped = 0
            admitted = 0
            j = 0
            while (j < len(queue) and len(active2) + len(active3) + len(starting) < self.max_active
                   and admitted < self.admit_per_poll):
                q = queue[j]
                if q.id not in footprint:
                    footprint[q.id] = self.backend.footprint(q)
                fp = footprint[q.id]
                if fp > self.budget:
                    raise ValueError(f"request {q.id} needs {fp} bytes, more than the whole budget")
                if self.in_use + fp <= self.budget:
                    q.handle = self.backend.create(q)
                    q.t_admit = self.clock() - t0
                    q.remaining = q.steps
                    self.in_use += fp
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    if isinstance(q.handle, concurrent.futures.Future):
                        starting.append(q)
                    else:
                        (active2 if q.dim == 2 else active3).append(q)
                    queue.pop(j)
                    admitted += 1
                    progressed = True
                else:
                    skipped += 1
                    if skipped > self.max_skip:
                        break
                    j += 1
            # launch every idle unit: a cohort per batched dimension, else
            # one unit per request
            cohorts = getattr(self.backend, "cohort_dims", (2,))
            for dim, members in ((2, active2), (3, active3)):
                if dim in cohorts:
                    if members and -dim not in flight:
                        k = min(self.chunk_for(dim), min(r.remaining for r in members))
                        flight[-dim] = (self.backend.launch(list(members), k), list(members), k)
                        chunks += 1
                        progressed = True
                    continue
                for r in members:
                    if r.id + 1 not in flight and self.backend.can_launch(r):
                        k = min(self.chunk_for(dim), r.remaining)
                        flight[r.id + 1] = (self.backend.launch([r], k), [r], k)
                        chunks += 1
                        progressed = True
            if not progressed:
                if not flight and i < len(pending):       # idle until the next arrival
                    wait = pending[i].t_arrive - (self.clock() - t0)
                    if wait > 0:
                        self._sleep(wait)
                else:
                    self.backend.idle()
        wall = self.clock() - t0
        # a time limit leaves requests unfinished: release them
        for q in starting:
            q.handle = q.handle.result()
        unfinished = active2 + active3 + starting
        if unfinished:
            self.backend.drain()
            for r in unfinished:
                self.backend.abandon(r)
                self.in_use -= footprint[r.id]
        if hasattr(self.backend, "close"):
            self.backend.close()
        lat = np.array([r.t_done - r.t_arrive for r in done]) if done else np.array([np.nan])
        cell_steps = float(sum(r.cells * r.steps for r in done))
        return {
            "completed": len(done), "submitted": len(requests), "wall_s": wall, "chunks": chunks,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(np.mean(lat)),
            "cell_steps_per_s": cell_steps / wall if wall > 0 else 0.0,
            "executed_cell_steps_per_s": executed / wall if wall > 0 else 0.0,
            "queued_or_active_at_end": len(requests) - len(done),
            "peak_hbm_bytes": self.peak_in_use, "done": done,
        }

    def chunk_for(self, dim: int) -> int:
        return self.chunk_3d if dim == 3 else self.chunk

    def _sleep(self, dt):
        if self.clock is time.perf_counter:
            time.sleep(min(dt, 0.05))
        elif hasattr(self.clock, "advance"):
            self.clock.advance(dt)


def requests_from_mix(mix) -> list:
    return [Request(id=m["id"], t_arrive=m["t_arrive"], dim=m["dim"], n=m["n"], k=tuple(m["k"]),
                    steps=m["steps"], amp=m["amp"], r=m["r"]) for m in mix]
