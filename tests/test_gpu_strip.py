"""Wave-strip form of the 2D column kernel (the default single-problem
path) against the CPU oracle and against the column-tile form.

The strip form streams each 64-column strip down a row segment; strips
near the x ends, segments near the y ends (the Pade band rows taken from
the table pass) and interior strips take different code, and the segment
lengths come from a per-geometry plan.  These cases put every form on the
oracle at sizes from one strip to many, for each sweep count the strip
form is built for.
"""
import numpy as np
import pytest

from gpu_util import check_fields, initial_fields, rel_l2, rel_l2_all, run_pair

pytestmark = pytest.mark.gpu

EH = ["ez", "hx", "hy"]


@pytest.mark.parametrize("n", [8, 9, 40, 49, 50, 97, 130, 301])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_strip_oracle_parity(n, lap):
    gf, of = run_pair(2, n, 0.5, 6, closure="paper" if n % 2 else "reflect", lap=lap, seed=100 + n)
    check_fields(gf, of)


@pytest.mark.parametrize("sweeps", [2, 3, 4, 6, 7, 8])
def test_strip_sweep_counts(sweeps):
    # every K the strip form is built for: the same K Chebyshev applications
    # as the column tiles (3), so the two agree to rounding
    from paper_2306_17263_amd import Problem
    n = 150
    init = initial_fields(2, n, 0.45, seed=sweeps)
    out = {}
    for shape in (3, 0):
        g = Problem(2, n, 0.45, sweeps=sweeps, tile_x=shape)
        for name in g.fields():
            g.set(name, init[name])
        g.step(4)
        out[shape] = {a: g.get(a) for a in EH}
        g.close()
    assert rel_l2_all(out[0], out[3], EH) <= 1e-13


@pytest.mark.parametrize("cfl", [0.2, 0.35, 0.58])
def test_strip_cfl(cfl):
    gf, of = run_pair(2, 120, cfl, 5, seed=7)
    check_fields(gf, of)


def test_strip_matches_tiles_and_oracle_large():
    # N = 2048 (many strips and segments): strips (0, 4) against the oracle
    # element by element and against the 128 x 4 column tiles (3), random
    # data, a few steps
    import oracle
    from paper_2306_17263_amd import Problem
    n, steps = 2048, 3
    init = initial_fields(2, n, 0.5, seed=21)
    out = {}
    for shape in (3, 0, 4):
        p = Problem(2, n, 0.5, tile_x=shape)
        for name in p.fields():
            p.set(name, init[name])
        p.step(steps)
        out[shape] = {a: p.get(a) for a in p.fields()}
        p.close()
    o = oracle.OracleProblem(2, n, 0.5)
    for name in init:
        o.set(name, init[name])
    o.step(steps)
    of = {a: o.get(a) for a in out[0]}
    for shape in (0, 4):
        check_fields(out[shape], of)
        assert rel_l2_all(out[shape], out[3], EH) <= 1e-13, shape
        assert rel_l2(out[shape]["lz"], out[3]["lz"]) <= 1e-10


def test_strip_many_rounds_large_grid():
    # N = 8192: the strip plan needs several rounds of the resident wave
    # slots; one step against the oracle (element by element) and the
    # 128 x 4 column tiles
    import oracle
    from paper_2306_17263_amd import Problem
    n = 8192
    init = initial_fields(2, n, 0.5, seed=8192)
    out = {}
    for shape in (3, 0):
        p = Problem(2, n, 0.5, tile_x=shape)
        for name in p.fields():
            p.set(name, init[name])
        p.step(1)
        out[shape] = {a: p.get(a) for a in EH}
        p.close()
    o = oracle.OracleProblem(2, n, 0.5)
    for name in init:
        o.set(name, init[name])
    o.step(1)
    check_fields(out[0], {a: o.get(a) for a in EH})
    assert rel_l2_all(out[0], out[3], EH) <= 1e-13


def test_batch_random_data_equals_alone():
    # seeded random fields (every operator mode), strips in the batch
    # against the same problems alone, bit for bit
    import torch
    from paper_2306_17263_amd import Batch, Problem
    ns = [8, 21, 50, 77, 130, 257]
    st = torch.cuda.Stream()
    b = Batch([{"n": n} for n in ns], stream=st, closure="paper", lap_mode="tracked")
    inits = [initial_fields(2, n, 0.5, seed=40 + n) for n in ns]
    for p, init in zip(b.problems, inits):
        for name in p.fields():
            p.set(name, init[name])
    b.step(5)
    for p, n, init in zip(b.problems, ns, inits):
        q = Problem(2, n, 0.5, stream=st, closure="paper", lap_mode="tracked")
        for name in q.fields():
            q.set(name, init[name])
        q.step(5)
        for a in EH:
            assert np.array_equal(p.get(a), q.get(a)), (n, a)
        q.close()
    b.close()
