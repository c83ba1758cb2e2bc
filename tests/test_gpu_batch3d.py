"""Batched 3D form (c4m_batch_create_from over 3D problems of different N):
every launch of the recorded 3D step runs once over all members.  Members'
fields equal, bit for bit, those of the same problems stepped alone, with
the carried and the discrete Laplacian and both closures; a member is
checked against the oracle too; graph replays equal direct launches; the
form refuses FP32-refined or PCG members and mixed dimensions."""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, check_fields, random_fields

pytestmark = pytest.mark.gpu

SIZES = (8, 20, 33, 64, 70)


def _members(sizes, stream, seed0, flags=0, **kw):
    from paper_2306_17263_amd import Problem
    probs, inits = [], []
    for i, n in enumerate(sizes):
        p = Problem(3, n, 0.4, stream=stream, flags=flags, **kw)
        f = random_fields(3, n, seed=seed0 + i, h_walls=True)
        for name in p.fields():
            p.set(name, f[name])
        probs.append(p)
        inits.append(f)
    return probs, inits


@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_batch3d_equals_alone(closure, lap):
    import torch
    from paper_2306_17263_amd import Batch
    st = torch.cuda.Stream()
    probs, inits = _members(SIZES, st, 30, closure=closure, lap_mode=lap)
    alone, _ = _members(SIZES, st, 30, closure=closure, lap_mode=lap)
    b = Batch.from_problems(probs, stream=st)
    for k in (3, 5):
        b.step(k)
        for p in alone:
            p.step(k)
        for p, q in zip(probs, alone):
            for name in p.fields():
                assert np.array_equal(p.get(name), q.get(name)), (p.n, name, k)
    # the smallest member against the oracle
    o = oracle.OracleProblem(3, SIZES[0], 0.4, 1.0, closure=CLOSURES[closure], lap_mode=LAPS[lap])
    for name, v in inits[0].items():
        if name in probs[0].fields():
            o.set(name, v)
    o.step(8)
    names = probs[0].fields()
    check_fields({a: probs[0].get(a) for a in names}, {a: o.get(a) for a in names})
    o.close()
    b.close()
    for p in probs + alone:
        p.close()


def test_batch3d_graph_and_direct_equal():
    import torch
    from paper_2306_17263_amd import FLAG_DIRECT, Batch
    st = torch.cuda.Stream()
    g_probs, _ = _members((12, 40, 27), st, 7)
    d_probs, _ = _members((12, 40, 27), st, 7, flags=FLAG_DIRECT)
    g = Batch.from_problems(g_probs, stream=st)
    d = Batch.from_problems(d_probs, stream=st)
    for steps in (2, 40, 3):
        g.step(steps)
        d.step(steps)
        for p, q in zip(g_probs, d_probs):
            for name in p.fields():
                assert np.array_equal(p.get(name), q.get(name)), (p.n, name)
    g.close()
    d.close()
    for p in g_probs + d_probs:
        p.close()


def test_batch3d_refusals():
    import torch
    from paper_2306_17263_amd import Batch, C4mError, Problem
    st = torch.cuda.Stream()
    for kw in (dict(precision="fp32_refined"), dict(solver="pcg")):
        probs = [Problem(3, 12, 0.4, stream=st, **kw), Problem(3, 16, 0.4, stream=st, **kw)]
        with pytest.raises(C4mError):
            Batch.from_problems(probs, stream=st)
        for p in probs:
            p.close()
    mixed = [Problem(3, 12, 0.4, stream=st), Problem(2, 16, 0.4, stream=st)]
    with pytest.raises(C4mError):
        Batch.from_problems(mixed, stream=st)
    for p in mixed:
        p.close()
