"""Captured runs of steps: c4m_step and c4m_batch_step replay HIP graphs of
up to 32 steps; with C4M_FLAG_PROFILE the same launches go to the stream
directly.  Every replay, with eager work (field reads, which synchronise)
between the replays, equals the direct launches bit for bit."""
import numpy as np
import pytest

from gpu_util import random_fields

pytestmark = pytest.mark.gpu


def _pair(dim, n, r, **kw):
    import torch
    from paper_2306_17263_amd import FLAG_PROFILE, Problem
    st = torch.cuda.Stream()
    f = random_fields(dim, n, seed=n + dim)
    g = Problem(dim, n, r, stream=st, **kw)                     # graphs
    d = Problem(dim, n, r, stream=st, flags=FLAG_PROFILE, **kw)  # direct launches
    for p in (g, d):
        for name in p.fields():
            p.set(name, f[name])
    return g, d


@pytest.mark.parametrize("dim,n,r,kw", [(2, 100, 0.5, {}), (2, 70, 0.5, {"solver": "pcg"}),
                                        (2, 90, 0.5, {"lap_mode": "discrete"}), (3, 20, 0.4, {})])
def test_step_graph_replays_equal_direct(dim, n, r, kw):
    g, d = _pair(dim, n, r, **kw)
    for rep, steps in enumerate((5, 5, 37, 1, 5)):             # 37 = one 32-step graph and a 5-step one
        g.step(steps)
        d.step(steps)
        for name in g.fields():
            assert np.array_equal(g.get(name), d.get(name)), (rep, name)
    assert g.info()["steps"] == d.info()["steps"] == 53
    g.close()
    d.close()


@pytest.mark.parametrize("tile_y", [0, 1])
def test_batch_graph_replays_equal_direct(tile_y):
    import torch
    from paper_2306_17263_amd import FLAG_PROFILE, Batch
    specs = [{"n": n} for n in (40, 130, 77)]
    st = torch.cuda.Stream()
    g = Batch(specs, stream=st, tile_y=tile_y)
    d = Batch(specs, stream=st, tile_y=tile_y, flags=FLAG_PROFILE)
    for b in (g, d):
        for p, s in zip(b.problems, specs):
            f = random_fields(2, s["n"], seed=s["n"])
            for name in p.fields():
                p.set(name, f[name])
    for rep, steps in enumerate((3, 3, 34)):
        g.step(steps)
        d.step(steps)
        for pg, pd in zip(g.problems, d.problems):
            for name in ("ez", "hx", "hy"):
                assert np.array_equal(pg.get(name), pd.get(name)), (rep, name)
    inf = d.info()
    cls = 7 if tile_y == 1 else 1                              # step / solve_e launches were timed
    assert inf["kernel_launches"][cls] == 40 and inf["kernel_ms"][cls] > 0
    g.check()
    d.check()
    g.close()
    d.close()


@pytest.mark.parametrize("dim,n", [(2, 70), (3, 20)])
def test_prepare_and_set_stream_change_nothing(dim, n):
    # graphs captured ahead by c4m_prepare on a set-up stream, the problem
    # then moved to another stream: same bits as a problem stepped plainly
    import torch
    from paper_2306_17263_amd import Problem
    init = random_fields(dim, n, seed=n)
    setup, work = torch.cuda.Stream(), torch.cuda.Stream()
    a = Problem(dim, n, 0.4, stream=setup)
    b = Problem(dim, n, 0.4, stream=work)
    for p in (a, b):
        for name in p.fields():
            p.set(name, init[name])
    a.prepare(70)
    a.prepare(6)
    a.set_stream(work)
    for k in (70, 6, 0, 33):
        a.step(k)
        b.step(k)
    for name in a.fields():
        assert np.array_equal(a.get(name), b.get(name)), name
    a.close()
    b.close()


@pytest.mark.parametrize("dim,n", [(2, 90), (3, 24)])
def test_direct_flag_equals_graphs(dim, n):
    # C4M_FLAG_DIRECT launches every step directly: same bits as graph replay
    import torch
    from paper_2306_17263_amd import FLAG_DIRECT, Problem
    init = random_fields(dim, n, seed=3 * n)
    st = torch.cuda.Stream()
    g = Problem(dim, n, 0.4, stream=st)
    d = Problem(dim, n, 0.4, stream=st, flags=FLAG_DIRECT)
    for p in (g, d):
        for name in p.fields():
            p.set(name, init[name])
    for k in (5, 40):
        g.step(k)
        d.step(k)
    for name in g.fields():
        assert np.array_equal(g.get(name), d.get(name)), name
    g.close()
    d.close()
