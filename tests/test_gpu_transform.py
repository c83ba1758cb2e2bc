"""The transform solver (C4M_SOLVER_TRANSFORM: M solved exactly by DST-I /
DCT-II matrix products on the FP64 matrix cores, Appendix A.2) against the
oracle, whose CG solve of M reaches 1e-15: 2D and 3D, both closures and both
Laplacian modes, sizes spanning several 64 x 64 product tiles with ragged
edges, random data with non-zero normal-H walls; and against the Chebyshev
solver on the same device.  FP32 refinement is refused with it."""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, check_fields, random_fields

pytestmark = pytest.mark.gpu


def _run(dim, n, r, steps, closure, lap, solver, seed, with_oracle=True):
    from paper_2306_17263_amd import Problem
    g = Problem(dim, n, r, closure=closure, lap_mode=lap, solver=solver)
    init = random_fields(dim, n, seed=seed, h_walls=True)
    for name in g.fields():
        g.set(name, init[name])
    g.step(steps)
    gf = {a: g.get(a) for a in g.fields()}
    g.close()
    of = None
    if with_oracle:
        o = oracle.OracleProblem(dim, n, r, 1.0, closure=CLOSURES[closure], lap_mode=LAPS[lap])
        for name in gf:
            o.set(name, init[name])
        o.step(steps)
        of = {a: o.get(a) for a in gf}
        o.close()
    return gf, of


@pytest.mark.parametrize("n", [8, 40, 97, 130])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_transform_2d_matches_oracle(n, closure, lap):
    gf, of = _run(2, n, 0.5, 4, closure, lap, "transform", seed=n)
    check_fields(gf, of)


@pytest.mark.parametrize("n", [8, 20, 33, 70])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_transform_3d_matches_oracle(n, closure, lap):
    gf, of = _run(3, n, 0.4, 3, closure, lap, "transform", seed=n)
    check_fields(gf, of)


@pytest.mark.parametrize("dim,n,r", [(2, 300, 0.5), (3, 96, 0.4)])
def test_transform_equals_chebyshev(dim, n, r):
    a, _ = _run(dim, n, r, 5, "paper", "tracked", "transform", seed=3, with_oracle=False)
    b, _ = _run(dim, n, r, 5, "paper", "tracked", "chebyshev", seed=3, with_oracle=False)
    check_fields(a, b)


def test_transform_refuses_fp32():
    from paper_2306_17263_amd import C4mError, Problem
    with pytest.raises(C4mError):
        Problem(2, 16, 0.5, solver="transform", precision="fp32_refined")
