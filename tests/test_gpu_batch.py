"""Batched form: every problem advanced inside the batch (persistent launches,
one HIP graph per step) equals the same problem advanced alone through the
single-problem path bit for bit, and the oracle to 1e-12."""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, initial_fields, rel_l2_all

pytestmark = pytest.mark.gpu


def _specs(seed=7):
    rng = np.random.default_rng(seed)
    ns = [9, 16, 33, 64, 70, 100, 129, 200]
    return [{"n": n, "k": (int(rng.integers(1, 5)), int(rng.integers(1, 5))),
             "amp": float(rng.uniform(0.5, 2))} for n in ns]


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
def test_batch_equals_alone_and_oracle(lap, closure):
    import torch
    from paper_2306_17263_amd import Batch, Problem
    specs = _specs()
    steps = 12
    st = torch.cuda.Stream()
    b = Batch(specs, stream=st, closure=closure, lap_mode=lap)
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
        assert rel_l2_all(gb, of, names) <= 1e-12, s["n"]
        assert p.info()["steps"] == steps
        alone.close()
    b.close()


def test_batch_rejects_mixed_settings():
    from paper_2306_17263_amd import Batch, C4mError
    with pytest.raises(C4mError):
        Batch([{"n": 16, "cfl": 0.5}, {"n": 20, "cfl": 0.4}])
