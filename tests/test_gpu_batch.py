"""Batched form: every problem advanced inside the batch equals the same
problem advanced alone through the single-problem path bit for bit, and the
oracle to the FP64 bar (1e-12 relative L2, every element within 1e-11 of the
field scale).

Bitwise equality holds because the batch and the single-problem kernels run
the same device functions on the same data and the library is built with
floating-point contraction fixed per source expression (-ffp-contract=on),
so a multiply-add is fused or not by the source, not by the kernel it is
inlined into."""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, check_fields, initial_fields, rel_l2_all

pytestmark = pytest.mark.gpu


def _specs(seed=7):
    rng = np.random.default_rng(seed)
    ns = [9, 16, 33, 64, 70, 100, 129, 200]
    return [{"n": n, "k": (int(rng.integers(1, 5)), int(rng.integers(1, 5))),
             "amp": float(rng.uniform(0.5, 2))} for n in ns]


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("tile_y", [0, 1])     # strips: one launch per stage / per step
def test_batch_equals_alone_and_oracle(lap, closure, tile_y):
    import torch
    from paper_2306_17263_amd import Batch, Problem
    specs = _specs()
    steps = 12
    st = torch.cuda.Stream()
    b = Batch(specs, stream=st, closure=closure, lap_mode=lap, tile_y=tile_y)
    inits = []
    for p, s in zip(b.problems, specs):
        init = initial_fields(2, s["n"], 0.5, k=s["k"], amp=s["amp"])
        inits.append(init)
        for name in p.fields():
            p.set(name, init[name])
    b.step(steps - 5)
    b.step(5)                                      # the graph is replayed across calls
    names = ["ez", "hx", "hy"]
    for p, s, init in zip(b.problems, specs, inits):
        # the batched form runs the single-problem kernels (the strip form by
        # default): bitwise equal to the problem run alone
        alone = Problem(2, s["n"], 0.5, stream=st, closure=closure, lap_mode=lap)
        for name in alone.fields():
            alone.set(name, init[name])
        alone.step(steps)
        o = oracle.OracleProblem(2, s["n"], 0.5, 1.0, closure=CLOSURES[closure], lap_mode=LAPS[lap])
        for name in alone.fields():
            o.set(name, init[name])
        o.step(steps)
        gb = {a: p.get(a) for a in names}
        ga = {a: alone.get(a) for a in names}
        of = {a: o.get(a) for a in names}
        for a in names:
            assert np.array_equal(gb[a], ga[a]), (s["n"], a)
        check_fields(gb, of)
        assert p.info()["steps"] == steps
        alone.close()
    b.check()
    b.close()


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("tile_y", [0, 1])
def test_batch_large_members_equal_alone(lap, tile_y):
    # members at the top of the batch workload's size range (N up to 768)
    # equal the problem run alone bit for bit, and the oracle
    import torch
    from paper_2306_17263_amd import Batch, Problem
    ns = [768, 64, 701, 400]
    steps = 6
    st = torch.cuda.Stream()
    b = Batch([{"n": n} for n in ns], stream=st, lap_mode=lap, tile_y=tile_y)
    inits = [initial_fields(2, n, 0.5, seed=500 + n) for n in ns]
    for p, init in zip(b.problems, inits):
        for name in p.fields():
            p.set(name, init[name])
    b.step(steps)
    names = ["ez", "hx", "hy"]
    for p, n, init in zip(b.problems, ns, inits):
        alone = Problem(2, n, 0.5, stream=st, lap_mode=lap)
        for name in alone.fields():
            alone.set(name, init[name])
        alone.step(steps)
        for a in names:
            assert np.array_equal(p.get(a), alone.get(a)), (n, a)
        alone.close()
        if n in (768, 64):
            o = oracle.OracleProblem(2, n, 0.5, 1.0, lap_mode=LAPS[lap])
            for name in alone.fields():
                o.set(name, init[name])
            o.step(steps)
            check_fields({a: p.get(a) for a in names}, {a: o.get(a) for a in names})
    b.close()


def test_batch_rejects_mixed_settings():
    from paper_2306_17263_amd import Batch, C4mError
    with pytest.raises(C4mError):
        Batch([{"n": 16, "cfl": 0.5}, {"n": 20, "cfl": 0.4}])


@pytest.mark.parametrize("shape,mult", [(1, 1), (2, 2), (0, 3), (3, 1)])
def test_batch_shapes_and_grid(shape, mult):
    import torch
    from paper_2306_17263_amd import Batch
    specs = _specs(11)[:5]
    st = torch.cuda.Stream()
    b = Batch(specs, stream=st, tile_x=shape, tile_y=mult)
    inits = []
    for p, s in zip(b.problems, specs):
        init = initial_fields(2, s["n"], 0.5, k=s["k"], amp=s["amp"])
        inits.append(init)
        for name in p.fields():
            p.set(name, init[name])
    b.step(6)
    for p, s, init in zip(b.problems, specs, inits):
        o = oracle.OracleProblem(2, s["n"], 0.5, 1.0)
        for name in p.fields():
            o.set(name, init[name])
        o.step(6)
        names = ["ez", "hx", "hy"]
        check_fields({a: p.get(a) for a in names}, {a: o.get(a) for a in names})
    b.close()


def test_autotune_batch_and_single(tmp_path, monkeypatch):
    monkeypatch.setenv("C4M_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2306_17263_amd import autotune
    r = autotune.tune_batch(_specs(3)[:4], steps=2)
    assert r["tile_x"] in (0, 1, 2) and r["tile_y"] in (1, 2)
    assert autotune.tune_batch(_specs(3)[:4], steps=2) == r          # served from the cache
    s = autotune.tune_single(96, steps=2)
    assert s["tile_x"] in autotune.SINGLE_SHAPES


def test_batch_check_quiet_and_forced_give_up():
    # single launch per step (tile_y 1): the default wait limit never gives
    # up on a normal run; a limit of one poll makes the Step 1 solve items
    # (taken while their x-lines still run) give up at once: the step
    # drains, nothing faults, and c4m_batch_check reports it once (then the
    # flag is clear)
    from paper_2306_17263_amd import Batch, C4mError, EDEVICE
    import torch
    specs = [{"n": 768}, {"n": 300}, {"n": 64}]
    st = torch.cuda.Stream()
    b = Batch(specs, stream=st, tile_y=1)
    for p, s in zip(b.problems, specs):
        init = initial_fields(2, s["n"], 0.5, seed=s["n"])
        for name in p.fields():
            p.set(name, init[name])
    b.step(3)
    b.check()
    b.close()
    b = Batch(specs, stream=st, tile_y=1, batch_wait_limit=1)
    for p, s in zip(b.problems, specs):
        init = initial_fields(2, s["n"], 0.5, seed=s["n"])
        for name in p.fields():
            p.set(name, init[name])
    b.step(2)
    with pytest.raises(C4mError) as ei:
        b.check()
    assert ei.value.status == EDEVICE
    b.check()
    b.close()


def test_full_batch_workload_sampled():
    """The whole 512-cavity workload the bench times (seed 2306, N 64..768,
    the default form), three steps; the largest, the smallest and a middle
    member against the oracle element by element, and the same members
    stepped alone bit for bit."""
    import torch
    from paper_2306_17263_amd import Batch, Problem
    from workloads import batch_mix, mode_fields
    specs = batch_mix(count=512)
    steps = 3
    st = torch.cuda.Stream()
    b = Batch([{"n": s["n"]} for s in specs], stream=st)
    order = sorted(range(len(specs)), key=lambda i: specs[i]["n"])
    picks = {order[0], order[len(order) // 2], order[-1]}
    inits = {}
    for i, (p, s) in enumerate(zip(b.problems, specs)):
        init = mode_fields(2, s["n"], s["k"], 0.0, s["r"] / s["n"] / 2, amp=s["amp"])
        for name in p.fields():
            p.set(name, init[name])
        if i in picks:
            inits[i] = init
    b.step(steps)
    names = ["ez", "hx", "hy"]
    for i in sorted(picks):
        s = specs[i]
        gf = {a: b.problems[i].get(a) for a in names}
        alone = Problem(2, s["n"], s["r"], stream=st)
        o = oracle.OracleProblem(2, s["n"], s["r"], 1.0)
        for name in alone.fields():
            alone.set(name, inits[i][name])
            o.set(name, inits[i][name])
        alone.step(steps)
        o.step(steps)
        for a in names:
            assert np.array_equal(gf[a], alone.get(a)), (s["n"], a)
        check_fields(gf, {a: o.get(a) for a in names})
        alone.close()
        o.close()
    b.check()
    b.close()
