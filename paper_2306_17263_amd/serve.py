"""Serving form: a continuous-batching request loop over the c4m stepper.

Requests (cavity simulations of different sizes and step counts) arrive over
time.  Each tick the server
  1. moves requests whose arrival time has passed into the queue;
  2. admits queued requests in arrival order while their device footprint
     fits the HBM budget and a slot is free (a request that does not fit
     waits; smaller later ones may pass it, up to `max_skip` of them);
  3. advances every active request: the active 2D requests together as one
     batch (persistent launches, re-formed only when membership changes),
     the 3D requests on side streams, by k = min(chunk, fewest remaining)
     steps so nobody overshoots; their work overlaps on the device;
  4. retires finished requests (fields copied out, memory released).
Latency of a request is completion minus arrival; the loop reports p50/p99
latency and completed cell-steps per second.  Fields stay resident on the
device from admission to retirement.

The backend is pluggable so the scheduling logic is testable on the CPU
(see tests/test_serve_cpu.py); DeviceBackend drives libc4m.so.
"""
from __future__ import annotations

import dataclasses
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

    @property
    def cells(self) -> int:
        return self.n ** self.dim


class DeviceBackend:
    """Requests on the GPU through libc4m.so (PyTorch for memory/streams)."""

    def __init__(self, n_side_streams: int = 2, settings: dict | None = None, keep_results: bool = False):
        import torch
        from .problem import make_config, workspace_bytes
        self.torch = torch
        self._make_config = make_config
        self._workspace_bytes = workspace_bytes
        self.settings = dict(settings or {})
        self.main = torch.cuda.Stream()
        self.side = [torch.cuda.Stream() for _ in range(n_side_streams)]
        self.keep_results = keep_results
        self._batch = None
        self._members = ()

    def footprint(self, req: Request) -> int:
        return self._workspace_bytes(self._make_config(req.dim, req.n, req.r, **self.settings))

    def create(self, req: Request):
        from workloads import mode_fields
        from .problem import Problem
        stream = self.main if req.dim == 2 else self.side[req.id % len(self.side)]
        p = Problem(req.dim, req.n, req.r, stream=stream, **self.settings)
        h = 1.0 / req.n
        init = mode_fields(req.dim, req.n, req.k, 0.0, req.r * h / 2, amp=req.amp)
        for name in p.fields():
            p.set(name, init[name])
        return p

    def step(self, active2d, active3d, k: int):
        from .batch import Batch
        key = tuple(id(r.handle) for r in active2d)
        if key != self._members:
            if self._batch is not None:
                self._batch.close()
            self._batch = Batch.from_problems([r.handle for r in active2d], stream=self.main) if active2d else None
            self._members = key
        if self._batch is not None:
            self._batch.step(k)
        for r in active3d:
            r.handle.step(k)

    def sync(self):
        self.torch.cuda.synchronize()

    def finish(self, req: Request):
        names = ["ez", "hx", "hy"] if req.dim == 2 else ["ex", "ey", "ez", "hx", "hy", "hz"]
        if self.keep_results:
            req.result = {a: req.handle.get(a) for a in names}
        if self._batch is not None and id(req.handle) in self._members:
            self._batch.close()                 # the batch references this problem
            self._batch = None
            self._members = ()
        req.handle.close()
        req.handle = None


class Server:
    def __init__(self, backend, hbm_budget: int, chunk: int = 50, max_active: int = 256, max_skip: int = 8,
                 clock=time.perf_counter):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.max_active = int(max_active)
        self.max_skip = int(max_skip)
        self.clock = clock
        self.in_use = 0
        self.peak_in_use = 0

    def run(self, requests, time_limit: float | None = None) -> dict:
        pending = sorted(requests, key=lambda q: q.t_arrive)
        queue, active, done = [], [], []
        footprint = {}
        t0 = self.clock()
        i = 0
        ticks = 0
        while i < len(pending) or queue or active:
            now = self.clock() - t0
            if time_limit is not None and now > time_limit:
                break
            while i < len(pending) and pending[i].t_arrive <= now:
                queue.append(pending[i])
                i += 1
            # admission by footprint, arrival order with bounded skipping
            skipped = 0
            j = 0
            while j < len(queue) and len(active) < self.max_active:
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
                    active.append(q)
                    queue.pop(j)
                else:
                    skipped += 1
                    if skipped > self.max_skip:
                        break
                    j += 1
            if not active:
                if i < len(pending):                # idle until the next arrival
                    wait = pending[i].t_arrive - (self.clock() - t0)
                    if wait > 0:
                        self._sleep(wait)
                continue
            k = min(self.chunk, min(r.remaining for r in active))
            a2 = [r for r in active if r.dim == 2]
            a3 = [r for r in active if r.dim == 3]
            self.backend.step(a2, a3, k)
            self.backend.sync()
            ticks += 1
            now = self.clock() - t0
            still = []
            for r in active:
                r.remaining -= k
                if r.remaining <= 0:
                    r.t_done = now
                    self.backend.finish(r)
                    self.in_use -= footprint[r.id]
                    done.append(r)
                else:
                    still.append(r)
            active = still
        wall = self.clock() - t0
        lat = np.array([r.t_done - r.t_arrive for r in done]) if done else np.array([np.nan])
        cell_steps = float(sum(r.cells * r.steps for r in done))
        return {
            "completed": len(done), "submitted": len(requests), "wall_s": wall, "ticks": ticks,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(np.mean(lat)),
            "cell_steps_per_s": cell_steps / wall if wall > 0 else 0.0,
            "peak_hbm_bytes": self.peak_in_use, "done": done,
        }

    def _sleep(self, dt):
        if self.clock is time.perf_counter:
            time.sleep(min(dt, 0.05))
        elif hasattr(self.clock, "advance"):
            self.clock.advance(dt)


def requests_from_mix(mix) -> list:
    return [Request(id=m["id"], t_arrive=m["t_arrive"], dim=m["dim"], n=m["n"], k=tuple(m["k"]),
                    steps=m["steps"], amp=m["amp"], r=m["r"]) for m in mix]
