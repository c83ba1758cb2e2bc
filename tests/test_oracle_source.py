"""Pins of the sourced oracle (Section 3.1, Table tab:spec; Method 2 ghosts,
eq:gst2), 2D TM with J = (0, 0, Jz).

* With zero sources and zero wall data it is the plain oracle's step.
* Its stencil of M (written out with numpy) equals the C oracle's.
* On a smooth exact solution driven by a current (workloads.driven, with
  non-zero Neumann data on every half-point wall) it converges at fourth
  order; each of the plausible slips (a dropped source or ghost term, the
  wall value of G_E) brings the order down to about two, and the source
  term as printed (rather than derived) does not converge at all.
* The wall reading: where Ez vanishes, Delta Ez = Z dJz/dt.
"""
import numpy as np
import pytest

from oracle import LAP_DISCRETE, LAP_TRACKED, OracleProblem
from oracle.source_oracle import SourcedTM, _ext, l9
from workloads import mode_fields
from workloads.driven import DrivenTM, _deriv

pytestmark = pytest.mark.filterwarnings("ignore")


def _zeros(n):
    e = np.zeros((1, n + 1, n + 1))
    w = [[np.zeros(n + 1), np.zeros(n + 1)] for _ in range(2)]
    d1 = {"jz": e, "jz_tt": e, "jz_lap": e, "jz_tt_lap": e, "hx_wall": w, "hy_wall": w}
    d2 = {"jz_t": e, "kx": np.zeros((1, n, n + 1)), "kx_lap": np.zeros((1, n, n + 1)),
          "ky": np.zeros((1, n + 1, n)), "ky_lap": np.zeros((1, n + 1, n)), "dhx_wall": w, "dhy_wall": w}
    return d1, d2


@pytest.mark.parametrize("lap", [LAP_TRACKED, LAP_DISCRETE])
def test_zero_sources_equal_plain_step(lap):
    n, r, z = 20, 0.5, 1.3
    f = mode_fields(2, n, (2, 3), 0.0, r / n / 2, z=z)
    s = SourcedTM(n, r, z, lap)
    o = OracleProblem(2, n, r, z, lap_mode=lap)
    for k in ("ez", "hx", "hy", "lz"):
        s.set(k, f[k])
        o.set(k, f[k])
    d1, d2 = _zeros(n)
    for _ in range(3):
        s.step(d1, d2)
        o.step(1)
    names = ("ez", "hx", "hy") + (("lz",) if lap == LAP_TRACKED else ())
    for k in names:
        a, b = s.get(k), o.get(k)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), k
    s.close()
    o.close()


@pytest.mark.parametrize("name,half_x,half_y", [("ez", False, False), ("hx", False, True), ("hy", True, False)])
def test_numpy_m_equals_c_oracle(name, half_x, half_y):
    n, r = 13, 0.5
    o = OracleProblem(2, n, r, 1.0)
    x = np.random.default_rng(5).standard_normal(o.shape(name))[0]
    alpha, beta = 1.0 + 2.0 / r ** 2, r * r / 24.0
    if not half_y:   # unknowns only: zeros on the node walls
        x[0, :] = x[-1, :] = 0.0
    if not half_x:
        x[:, 0] = x[:, -1] = 0.0
    mine = alpha * x - beta * l9(_ext(x, half_x, half_y))
    ref = o.apply_m(name, x[None])[0]
    sl = (slice(None) if half_y else slice(1, -1), slice(None) if half_x else slice(1, -1))
    np.testing.assert_allclose(mine[sl], ref[sl], rtol=0, atol=1e-13)
    o.close()


def _run(drv, n, r, T, lap, mutate=None):
    h = 1.0 / n
    ht = r * h
    steps = int(round(T / ht))
    s = SourcedTM(n, r, drv.z, lap)
    f0 = drv.fields(n, 0.0, ht / 2)
    for k in ("ez", "hx", "hy", "lz"):
        s.set(k, f0[k])
    for m in range(steps):
        d1, d2 = drv.step1_data(n, (m + 0.5) * ht), drv.step2_data(n, (m + 1) * ht)
        if mutate:
            mutate(d1, d2)
        s.step(d1, d2)
    fe = drv.fields(n, steps * ht, (steps + 0.5) * ht)
    err = max(np.max(np.abs(s.get(k) - fe[k])) for k in ("ez", "hx", "hy"))
    s.close()
    return err


def _rates(drv, lap, mutate=None, ns=(16, 32, 64)):
    errs = [_run(drv, n, 0.5, 0.25, lap, mutate) for n in ns]
    return errs, [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("z", [1.0, 1.7])
@pytest.mark.parametrize("lap", [LAP_TRACKED, LAP_DISCRETE])
def test_driven_cavity_fourth_order(z, lap):
    errs, rates = _rates(DrivenTM(z=z), lap)
    assert min(rates) >= 4.0, (errs, rates)
    assert errs[-1] < 5e-8


def _drop(*keys):
    def mutate(d1, d2):
        for d in (d1, d2):
            for k in keys:
                if k in d:
                    v = d[k]
                    d[k] = [[0 * a for a in w] for w in v] if isinstance(v, list) else 0 * v
    return mutate


@pytest.mark.parametrize("keys", [("jz_tt", "jz_tt_lap"), ("kx", "kx_lap", "ky", "ky_lap"), ("jz_lap", "jz_tt_lap"),
                                  ("dhx_wall",), ("hy_wall",), ("jz_t",)])
def test_each_source_term_is_needed(keys):
    """Dropping any one group of source data loses the fourth order."""
    _, rates = _rates(DrivenTM(), LAP_TRACKED, _drop(*keys))
    assert rates[-1] < 3.0, (keys, rates)


def test_third_derivative_ghost_term_is_needed():
    drv = DrivenTM()

    def mutate(d1, d2):
        for d, keys in ((d1, ("hx_wall", "hy_wall")), (d2, ("dhx_wall", "dhy_wall"))):
            for k in keys:
                d[k] = [[w[0], 0 * w[1]] for w in d[k]]

    _, rates = _rates(drv, LAP_TRACKED, mutate)
    assert rates[-1] < 3.0, rates


def test_printed_source_term_does_not_converge():
    """The printed P(J) (Z(-J - grad div J + d2J/dt2), with h_t^2/24 in front
    of it in F) in place of the derived F_J = -Z (J + (h_t^2/24) d2J/dt2):
    fed through the same inputs (jz -> (h_t^2/24) J, jz_tt -> -J_tt) the
    error stays of the size of the solution."""
    r = 0.5

    def make(n):
        ht2 = (r / n) ** 2 / 24.0

        def mutate(d1, d2):
            d1["jz"], d1["jz_tt"] = ht2 * d1["jz"], -d1["jz_tt"]
            d1["jz_lap"], d1["jz_tt_lap"] = ht2 * d1["jz_lap"], -d1["jz_tt_lap"]
        return mutate

    drv = DrivenTM()
    errs = [_run(drv, n, r, 0.25, LAP_TRACKED, make(n)) for n in (16, 32)]
    assert min(errs) > 1e-2, errs


def test_wall_laplacian_of_ez_is_z_djz_dt():
    """Where Ez vanishes (a PEC wall), d2Ez/dt2 = 0, so the wave equation
    with a current gives Delta Ez = Z dJz/dt there."""
    drv = DrivenTM(z=1.4)
    t = 0.37
    xs = np.linspace(0.0, 1.0, 11)
    for yw in (0.0, 1.0):
        lap = drv._s(0, t) * (_deriv(drv.a, 2, xs) * _deriv(drv.b, 0, yw) + _deriv(drv.a, 0, xs) * _deriv(drv.b, 2, yw))
        st, sd = drv._s(0, t), drv._s(2, t)
        a = _deriv(drv.a, 2, xs) * _deriv(drv.b, 0, yw) + _deriv(drv.a, 0, xs) * _deriv(drv.b, 2, yw)
        bb = _deriv(drv.a, 0, xs) * _deriv(drv.b, 0, yw)
        jz_t = (st * a - sd * bb) / drv.z
        np.testing.assert_allclose(lap, drv.z * jz_t, rtol=0, atol=1e-12)
