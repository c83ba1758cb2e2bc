"""Edge cases of the GPU stepper: zero data, linearity of the step map at a
large size (a property that holds at any size), and oracle parity on a
large grid (zero steps: test_gpu_boundary.py)."""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, check_fields, initial_fields, rel_l2_all

pytestmark = pytest.mark.gpu


def _problem(dim, n, cfl, fields, **kw):
    from paper_2306_17263_amd import Problem
    p = Problem(dim, n, cfl, **kw)
    for name in p.fields():
        p.set(name, fields[name])
    return p


@pytest.mark.parametrize("dim,n,cfl", [(2, 40, 0.5), (3, 12, 0.4)])
def test_zero_data_stays_zero(dim, n, cfl):
    init = initial_fields(dim, n, cfl, k=(1, 1) if dim == 2 else (1, 1, 1))
    zero = {a: np.zeros_like(v) for a, v in init.items()}
    p = _problem(dim, n, cfl, zero)
    p.step(5)
    for name in p.fields():
        assert not np.any(p.get(name)), name
    p.close()


def test_step_map_is_linear_large():
    # S(a u + b v) = a S(u) + b S(v) up to rounding, at N = 1024
    n, cfl = 1024, 0.5
    u = initial_fields(2, n, cfl, k=(3, 5))
    v = initial_fields(2, n, cfl, k=(7, 2))
    a, b = 0.75, -1.25
    w = {k: a * u[k] + b * v[k] for k in u}
    out = {}
    for tag, f in (("u", u), ("v", v), ("w", w)):
        p = _problem(2, n, cfl, f)
        p.step(4)
        out[tag] = {x: p.get(x) for x in ("ez", "hx", "hy")}
        p.close()
    comb = {x: a * out["u"][x] + b * out["v"][x] for x in out["w"]}
    assert rel_l2_all(out["w"], comb, ["ez", "hx", "hy"]) <= 1e-14


def test_large_grid_parity():
    n, cfl, steps = 4096, 0.5, 1
    init = initial_fields(2, n, cfl, k=(9, 4))
    p = _problem(2, n, cfl, init)
    p.step(steps)
    o = oracle.OracleProblem(2, n, cfl, 1.0, closure=CLOSURES["paper"], lap_mode=LAPS["tracked"])
    for name in p.fields():
        o.set(name, init[name])
    o.step(steps)
    names = ["ez", "hx", "hy"]
    check_fields({x: p.get(x) for x in p.fields()}, {x: o.get(x) for x in p.fields()})
    p.close()
