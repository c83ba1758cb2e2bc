"""PCG form of the compact solve (Jacobi-preconditioned CG with device
reductions, the solver the paper names for the SPD systems): parity with the
oracle, iteration statistics, the non-convergence flag and run-to-run
determinism of the reductions."""
import numpy as np
import pytest

from gpu_util import check_fields, initial_fields, rel_l2_all, run_pair

pytestmark = pytest.mark.gpu

EH2 = ["ez", "hx", "hy"]
EH3 = ["ex", "ey", "ez", "hx", "hy", "hz"]


@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("n", [33, 130])
def test_pcg_parity_2d(closure, lap, n):
    gf, of = run_pair(2, n, 0.5, 12, closure=closure, lap=lap, k=(3, 2), solver="pcg")
    check_fields(gf, of)


def test_pcg_random_data_2d():
    gf, of = run_pair(2, 77, 0.45, 6, seed=1234, solver="pcg")
    check_fields(gf, of)


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("n", [8, 13])
def test_pcg_parity_3d(lap, n):
    gf, of = run_pair(3, n, 0.4, 4, lap=lap, k=(2, 3, 4), solver="pcg")
    check_fields(gf, of)


def _problem(n=64, steps=4, **kw):
    from paper_2306_17263_amd import Problem
    init = initial_fields(2, n, 0.5, k=(2, 3))
    p = Problem(2, n, 0.5, solver="pcg", **kw)
    for name in p.fields():
        p.set(name, init[name])
    p.step(steps)
    return p


def test_pcg_statistics():
    p = _problem()
    inf = p.info()
    assert 1 <= inf["last_iters"] <= 16
    assert inf["max_iters"] >= inf["last_iters"]
    assert inf["last_rel_residual"] <= 1e-14
    assert inf["noconv"] == 0
    p.close()


def test_pcg_noconv_flag():
    # one iteration cannot reach 1e-14: the solve ends and flags it
    p = _problem(max_iter=1, rtol=1e-15)
    inf = p.info()
    assert inf["noconv"] == 1
    assert inf["last_iters"] == 1
    p.close()


def test_pcg_deterministic_and_matches_chebyshev():
    from paper_2306_17263_amd import Problem
    a = _problem(n=96, steps=6)
    b = _problem(n=96, steps=6)
    for name in EH2:
        assert np.array_equal(a.get(name), b.get(name)), name
    init = initial_fields(2, 96, 0.5, k=(2, 3))
    c = Problem(2, 96, 0.5)
    for name in c.fields():
        c.set(name, init[name])
    c.step(6)
    assert rel_l2_all({x: a.get(x) for x in EH2}, {x: c.get(x) for x in EH2}, EH2) <= 1e-12
    for p in (a, b, c):
        p.close()
