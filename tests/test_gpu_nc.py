"""The non-compact comparison scheme NC on the device (c4m_config.scheme =
C4M_SCHEME_NC) against its oracle: every element within 1e-12 relative of
the field scale after the same steps, on grids from one tile to many, mode
and random data, Z != 1, CFL at its bound; the configuration checks."""
import numpy as np
import pytest

from gpu_util import check_fields, random_fields
from oracle.nc_oracle import NCProblem
from workloads import mode_fields

pytestmark = pytest.mark.gpu

EH = ["ez", "hx", "hy"]


def _pair(n, r, steps, init, z=1.0):
    from paper_2306_17263_amd import Problem
    g = Problem(2, n, r, z=z, scheme="nc")
    o = NCProblem(n, r, z)
    for name in EH:
        g.set(name, init[name])
        o.set(name, init[name])
    g.step(steps)
    o.step(steps)
    out = ({a: g.get(a) for a in EH}, {a: o.get(a) for a in EH})
    g.close()
    return out


@pytest.mark.parametrize("n", [8, 33, 96, 130, 301])
def test_nc_mode_parity(n):
    r = 0.5
    init = mode_fields(2, n, (3, 2), 0.0, r / n / 2, with_laplacian=False)
    gf, of = _pair(n, r, 20, init)
    check_fields(gf, of, lap_tol=None)


@pytest.mark.parametrize("n", [9, 64, 200])
def test_nc_random_parity(n):
    init = random_fields(2, n, seed=n, h_walls=True)
    gf, of = _pair(n, 0.45, 8, init, z=1.7)
    check_fields(gf, of, lap_tol=None)


def test_nc_long_run_and_cfl_bound():
    n, r = 64, 6 / (7 * np.sqrt(2))
    init = mode_fields(2, n, (2, 2), 0.0, r / n / 2, with_laplacian=False)
    gf, of = _pair(n, r, 300, init)
    check_fields(gf, of, lap_tol=None)


def test_nc_configuration_checks():
    from paper_2306_17263_amd import C4mError, EINVAL, EUNSTABLE, Batch, Problem
    with pytest.raises(C4mError) as ei:
        Problem(2, 32, 0.61, scheme="nc")
    assert ei.value.status == EUNSTABLE
    for kw in ({"precision": "fp32_refined"},):
        with pytest.raises(C4mError) as ei:
            Problem(2, 32, 0.5, scheme="nc", **kw)
        assert ei.value.status == EINVAL
    with pytest.raises(C4mError) as ei:
        Problem(3, 16, 0.4, scheme="nc")
    assert ei.value.status == EINVAL
    with pytest.raises(C4mError) as ei:
        Batch([{"n": 16}, {"n": 20}], scheme="nc")
    assert ei.value.status == EINVAL
    p = Problem(2, 32, 0.5, scheme="nc")
    assert p.fields() == EH
    p.close()
