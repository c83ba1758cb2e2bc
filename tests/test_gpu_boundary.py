"""Boundary data and failure reporting at the C ABI.

* Normal H on the PEC walls is constant in time (eq:BC_H) and enters the
  source conditioning of Step 1 as the wall value of the node-direction
  stencil: non-zero wall values, given through c4m_set_field (whole array)
  or c4m_set_boundary (one wall plane), match the oracle holding the same
  values, 2D and 3D, and stay unchanged by stepping.
* Tangential E and l vanish on the walls (eq:bc_E=0): non-zero values are
  rejected with EINVAL (host and device sources) and leave the state as it
  was; rounding-level values are stored as zero.
* c4m_step(p, 0) changes nothing, the carried Laplacian included.
* C4M_FLAG_CHECK_FINITE reports ENONFINITE once the scheme, run above its
  stability bound (r = 1/sqrt 2, Table cfl), has overflowed; a stable run is
  not flagged.
"""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, check_fields, random_fields

pytestmark = pytest.mark.gpu


def _pair(dim, n, r, closure="paper", lap="tracked", **kw):
    from paper_2306_17263_amd import Problem
    g = Problem(dim, n, r, closure=closure, lap_mode=lap, **kw)
    o = oracle.OracleProblem(dim, n, r, 1.0, closure=CLOSURES[closure], lap_mode=LAPS[lap])
    return g, o


def _wall_plane(arr, axis, side):
    sl = [slice(None)] * 3
    sl[2 - axis] = -1 if side else 0
    return arr[tuple(sl)]


@pytest.mark.parametrize("dim,n,r", [(2, 40, 0.5), (2, 97, 0.5), (3, 12, 0.4), (3, 60, 0.4)])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_normal_h_walls_via_set_field(dim, n, r, lap):
    f = random_fields(dim, n, seed=31 * n + dim, h_walls=True)
    g, o = _pair(dim, n, r, lap=lap)
    for name in g.fields():
        g.set(name, f[name])
        o.set(name, f[name])
    g.step(4)
    o.step(4)
    gf = {a: g.get(a) for a in g.fields()}
    check_fields(gf, {a: o.get(a) for a in g.fields()})
    for name in gf:
        if name[0] == "h":
            ax = "xyz".index(name[1])
            for side in (0, 1):
                assert np.array_equal(_wall_plane(gf[name], ax, side), _wall_plane(f[name], ax, side)), name
    g.close()


@pytest.mark.parametrize("dim,n,r", [(2, 50, 0.5), (3, 16, 0.4)])
@pytest.mark.parametrize("device_src", [False, True])
def test_normal_h_walls_via_set_boundary(dim, n, r, device_src):
    import torch
    f = random_fields(dim, n, seed=5 + n)                    # zero normal H on the walls
    g, o = _pair(dim, n, r)
    for name in g.fields():
        g.set(name, f[name])
    rng = np.random.default_rng(n)
    for name in [a for a in f if a[0] == "h"]:
        ax = "xyz".index(name[1])
        for side in (0, 1):
            plane = rng.normal(size=_wall_plane(f[name], ax, side).shape)
            sl = [slice(None)] * 3
            sl[2 - ax] = -1 if side else 0
            f[name][tuple(sl)] = plane
            vals = torch.from_numpy(np.ascontiguousarray(plane)).cuda() if device_src else plane
            g.set_boundary(name, 2 * ax + side, vals)
    for name in g.fields():
        o.set(name, f[name])
    for name in [a for a in f if a[0] == "h"]:
        assert np.array_equal(g.get(name), f[name]), name
    g.step(3)
    o.step(3)
    check_fields({a: g.get(a) for a in g.fields()}, {a: o.get(a) for a in g.fields()})
    g.close()


@pytest.mark.parametrize("device_src", [False, True])
def test_nonzero_tangential_e_rejected(device_src):
    import torch
    from paper_2306_17263_amd import C4mError, EINVAL, Problem
    n = 24
    f = random_fields(2, n, seed=3)
    p = Problem(2, n, 0.5)
    for name in p.fields():
        p.set(name, f[name])
    before = {a: p.get(a) for a in p.fields()}
    for name in ("ez", "lz"):
        bad = f[name].copy()
        bad[0, 0, 5] = 0.25                                   # y = 0 wall
        src = torch.from_numpy(bad).cuda() if device_src else bad
        with pytest.raises(C4mError) as ei:
            p.set(name, src)
        assert ei.value.status == EINVAL
        # rounding-level wall values are accepted and stored as zero
        tiny = f[name].copy()
        tiny[0, -1, 3] = 1e-16 * np.max(np.abs(tiny))
        p.set(name, torch.from_numpy(tiny).cuda() if device_src else tiny)
        assert p.get(name)[0, -1, 3] == 0.0
    for name in p.fields():
        assert np.array_equal(p.get(name), before[name]), name
    p.close()


def test_set_boundary_rules():
    from paper_2306_17263_amd import C4mError, EINVAL, Problem
    n = 20
    p = Problem(3, n, 0.4)
    # Ex lives on the y and z walls (tangential): zeros are fine, others not
    zero = np.zeros((n + 1, n))                               # Ex without its y axis: (nz, nx)
    p.set_boundary("ex", 2, zero)
    with pytest.raises(C4mError) as ei:
        p.set_boundary("ex", 2, zero + 1.0)
    assert ei.value.status == EINVAL
    for name, face in (("ex", 0), ("hx", 2), ("hz", 1), ("ey", 7)):
        with pytest.raises(C4mError) as ei:
            shp = list(p.shape(name))
            del shp[2 - min(face // 2, 2)]
            p.set_boundary(name, face, np.zeros(shp))
        assert ei.value.status == EINVAL, (name, face)
    p.close()


@pytest.mark.parametrize("dim,n,r", [(2, 64, 0.5), (3, 16, 0.4)])
def test_zero_steps_is_identity(dim, n, r):
    from paper_2306_17263_amd import Problem
    f = random_fields(dim, n, seed=3)
    p = Problem(dim, n, r)
    for name in p.fields():
        p.set(name, f[name])
    before = {x: p.get(x) for x in p.fields()}
    p.step(0)
    for name in p.fields():
        assert np.array_equal(p.get(name), before[name]), name
    assert p.info()["steps"] == 0
    p.close()


def test_nonfinite_flag_above_stability_bound():
    # r = 1/sqrt(2) is above the bound (Table cfl, last row): the modes that
    # grow overflow FP64 within a few thousand steps; the check after the
    # call finds the NaN/Inf and the flag stays set
    from paper_2306_17263_amd import C4mError, ENONFINITE, Problem, FLAG_ALLOW_ANY_CFL, FLAG_CHECK_FINITE
    n = 32
    r = 1 / np.sqrt(2)
    f = random_fields(2, n, seed=9)
    p = Problem(2, n, r, flags=FLAG_ALLOW_ANY_CFL | FLAG_CHECK_FINITE)
    for name in p.fields():
        p.set(name, f[name])
    p.step(10)                                                # still finite
    assert p.info()["nonfinite"] == 0
    with pytest.raises(C4mError) as ei:
        p.step(6000)
    assert ei.value.status == ENONFINITE
    assert p.info()["nonfinite"] == 1
    p.close()


def test_finite_check_quiet_when_stable():
    from paper_2306_17263_amd import FLAG_CHECK_FINITE, Problem
    n = 32
    f = random_fields(2, n, seed=9)
    p = Problem(2, n, 0.5, flags=FLAG_CHECK_FINITE)
    for name in p.fields():
        p.set(name, f[name])
    p.step(500)
    assert p.info()["nonfinite"] == 0
    p.close()
