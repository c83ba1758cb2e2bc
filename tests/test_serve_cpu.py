"""Scheduling logic of the serving loop on the CPU: a fake backend (the
oracle for the fields, a virtual clock for time, one serial device on which
launched chunks queue up) behind the same interface as the device backend."""
import numpy as np
import pytest

import oracle
from paper_2306_17263_amd.serve import Request, Server, requests_from_mix
from workloads import mode_fields, serving_arrivals


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt


class FakeBackend:
    """Oracle problems; every step advances the virtual clock by its cost."""

    def __init__(self, clock, cost_per_cell_step=1e-9, bytes_per_cell=64, cohort_dims=(2,)):
        self.clock = clock
        self.cohort_dims = cohort_dims
        self.cost = cost_per_cell_step
        self.bpc = bytes_per_cell
        self.steps_done = {}
        self.live = set()
        self.max_live = 0
        self.device_free = 0.0
        self.outstanding = set()
        self.launches = 0

    def footprint(self, req):
        return req.cells * self.bpc

    def create(self, req):
        p = oracle.OracleProblem(req.dim, req.n, req.r)
        h = 1.0 / req.n
        for name, v in mode_fields(req.dim, req.n, req.k, 0.0, req.r * h / 2, amp=req.amp).items():
            p.set(name, v)
        self.steps_done[req.id] = 0
        self.live.add(req.id)
        self.max_live = max(self.max_live, len(self.live))
        return p

    def launch(self, reqs, k):
        assert k >= 1
        assert len({r.dim for r in reqs}) == 1 and (reqs[0].dim in self.cohort_dims or len(reqs) == 1)
        for r in reqs:
            assert self.steps_done[r.id] + k <= r.steps          # never overshoots
            r.handle.step(k)
            self.steps_done[r.id] += k
        start = max(self.device_free, self.clock())
        self.device_free = start + self.cost * k * sum(r.cells for r in reqs)
        self.outstanding.add(self.device_free)
        self.launches += 1
        return self.device_free

    def can_launch(self, req):
        return True

    def done(self, token):
        if self.clock() >= token:
            self.outstanding.discard(token)
            return True
        return False

    def idle(self):
        if self.outstanding:
            self.clock.t = max(self.clock.t, min(self.outstanding))
        else:
            self.clock.advance(1e-6)

    def drain(self):
        self.clock.t = max([self.clock.t] + list(self.outstanding))
        self.outstanding.clear()

    def abandon(self, req):
        self.live.discard(req.id)
        req.handle = None

    def finish(self, req):
        names = ["ez", "hx", "hy"] if req.dim == 2 else ["ex", "ey", "ez", "hx", "hy", "hz"]
        req.result = {a: req.handle.get(a) for a in names}
        self.live.discard(req.id)
        req.handle = None


def _mix(count=12, seed=3):
    mix = serving_arrivals(count=count, seed=seed, rate=50.0, n2=(8, 24), n3=(8, 10), steps=(3, 12))
    return requests_from_mix(mix)


def test_all_requests_complete_with_exact_step_counts():
    clock = VirtualClock()
    be = FakeBackend(clock)
    reqs = _mix()
    out = Server(be, hbm_budget=10 ** 9, chunk=4, clock=clock).run(reqs)
    assert out["completed"] == len(reqs)
    for r in out["done"]:
        assert be.steps_done[r.id] == r.steps
        assert r.t_done >= r.t_admit >= r.t_arrive - 1e-12


def test_admission_respects_the_budget():
    clock = VirtualClock()
    be = FakeBackend(clock)
    reqs = _mix(16)
    budget = max(be.footprint(r) for r in reqs) * 2
    srv = Server(be, hbm_budget=budget, chunk=3, clock=clock)
    out = srv.run(reqs)
    assert out["completed"] == len(reqs)
    assert srv.peak_in_use <= budget
    assert be.max_live >= 1


def test_request_larger_than_budget_is_refused():
    clock = VirtualClock()
    be = FakeBackend(clock)
    reqs = _mix(3)
    with pytest.raises(ValueError):
        Server(be, hbm_budget=10, clock=clock).run(reqs)


def test_result_in_the_mix_equals_result_alone():
    clock = VirtualClock()
    be = FakeBackend(clock)
    reqs = _mix(8, seed=5)
    out = Server(be, hbm_budget=10 ** 9, chunk=5, clock=clock).run(reqs)
    for r in out["done"]:
        alone = oracle.OracleProblem(r.dim, r.n, r.r)
        h = 1.0 / r.n
        for name, v in mode_fields(r.dim, r.n, r.k, 0.0, r.r * h / 2, amp=r.amp).items():
            alone.set(name, v)
        alone.step(r.steps)
        for a, v in r.result.items():
            assert np.array_equal(v, alone.get(a)), (r.id, a)


def test_latency_percentiles_reported():
    clock = VirtualClock()
    out = Server(FakeBackend(clock), hbm_budget=10 ** 9, chunk=4, clock=clock).run(_mix(10))
    assert 0 <= out["p50_latency_s"] <= out["p99_latency_s"]
    assert out["cell_steps_per_s"] > 0


def test_units_progress_independently():
    # a long 3D request admitted first does not hold back 2D requests that
    # arrive after it: their chunks interleave with its chunks on the device
    from paper_2306_17263_amd.serve import Request
    clock = VirtualClock()
    be = FakeBackend(clock)
    reqs = [Request(id=0, t_arrive=0.0, dim=3, n=10, k=(1, 1, 1), steps=40, r=0.4),
            Request(id=1, t_arrive=1e-7, dim=2, n=12, k=(1, 2), steps=4),
            Request(id=2, t_arrive=2e-7, dim=2, n=16, k=(2, 1), steps=6)]
    out = Server(be, hbm_budget=10 ** 9, chunk=2, clock=clock).run(reqs)
    assert out["completed"] == 3
    t = {r.id: r.t_done for r in out["done"]}
    assert t[1] < t[0] and t[2] < t[0]
    assert be.steps_done == {0: 40, 1: 4, 2: 6}


def test_time_limit_releases_unfinished_requests():
    clock = VirtualClock()
    be = FakeBackend(clock, cost_per_cell_step=1e-6)
    reqs = _mix(12)
    srv = Server(be, hbm_budget=10 ** 9, chunk=2, clock=clock)
    out = srv.run(reqs, time_limit=1e-3)
    assert out["completed"] < len(reqs)
    assert srv.in_use == 0 and not be.live
    assert out["queued_or_active_at_end"] == len(reqs) - out["completed"]


def test_3d_cohort_exact_steps_and_results():
    # 3D requests batched as a cohort (as the device backend does) reach
    # exactly their step counts and the result each would reach alone
    clock = VirtualClock()
    be = FakeBackend(clock, cohort_dims=(2, 3))
    reqs = _mix(10, seed=9)
    out = Server(be, hbm_budget=10 ** 9, chunk=4, chunk_3d=3, clock=clock).run(reqs)
    assert out["completed"] == len(reqs)
    for r in out["done"]:
        assert be.steps_done[r.id] == r.steps
        alone = oracle.OracleProblem(r.dim, r.n, r.r)
        h = 1.0 / r.n
        for name, v in mode_fields(r.dim, r.n, r.k, 0.0, r.r * h / 2, amp=r.amp).items():
            alone.set(name, v)
        alone.step(r.steps)
        for a, v in r.result.items():
            assert np.array_equal(v, alone.get(a)), (r.id, a)
