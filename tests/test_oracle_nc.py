"""Pins of the NC comparison scheme's oracle (Section 5.2, stencil K4 at
a = 0, one-sided fourth-order rows next to the walls).

* The staggered derivative rows: the interior K4 row is exact on quartics
  and the one-sided row on cubics (their Taylor moments), not beyond;
  smooth data converge at fourth order.
* Table cfl, NC column (k = 2, h = 1/64, T = 4/sqrt 2): the five printed
  mean absolute errors within 3 % (same error-metric reading as the C4
  column), and r = 1/sqrt 2 blows up.
* Table conv_rates, NC column (k = 2, r = 5/(6 sqrt 2), T = 1/sqrt 2): the
  printed rates 1.98 (N = 64) and 1.98 (N = 128) within 0.05.
"""
import os

import numpy as np
import pytest

from oracle.nc_oracle import NCProblem, staggered_derivative
from workloads import mode_fields


def _points(m, node_inputs):
    """Input abscissae of one line of m inputs and the outputs between
    consecutive inputs (h = 1)."""
    xin = np.arange(m) + (0.0 if node_inputs else 0.5)
    return xin, xin[:-1] + 0.5


@pytest.mark.parametrize("m", [8, 13, 40])
def test_rows_exact_on_polynomials(m):
    rng = np.random.default_rng(m)
    xin, xout = _points(m, node_inputs=True)
    for deg, interior_only in ((3, False), (4, True)):
        c = rng.normal(size=deg + 1)
        got = staggered_derivative(np.polyval(c, xin)[None, :], m - 1)[0]
        ref = np.polyval(np.polyder(c), xout)
        scale = 1 + np.max(np.abs(ref))
        if interior_only:
            # the one-sided rows (first and last output) are not exact on quartics
            assert np.max(np.abs(got[1:-1] - ref[1:-1])) <= 1e-9 * scale
            assert np.max(np.abs(got[[0, -1]] - ref[[0, -1]])) > 1e-6
        else:
            assert np.max(np.abs(got - ref)) <= 1e-9 * scale
    # quintics break the interior row too
    got = staggered_derivative((xin ** 5)[None, :], m - 1)[0]
    assert np.max(np.abs(got[1:-1] - 5 * xout[1:-1] ** 4)) > 1e-3


def test_truncation_orders_on_smooth_data():
    # interior K4 rows: fourth order; the one-sided wall rows: third order
    # (their fourth Taylor moment does not vanish)
    inner, wall = [], []
    for n in (32, 64, 128, 256):
        h = 1.0 / n
        xin = (np.arange(n) + 0.5) * h                  # half points -> interior nodes
        got = staggered_derivative(np.cos(3 * xin)[None, :], n - 1)[0] / h
        err = np.abs(got + 3 * np.sin(3 * np.arange(1, n) * h))
        inner.append(np.max(err[1:-1]))
        wall.append(np.max(err[[0, -1]]))
    r_in = np.log2(np.array(inner[:-1]) / np.array(inner[1:]))
    r_wall = np.log2(np.array(wall[:-1]) / np.array(wall[1:]))
    assert np.all(np.abs(r_in - 4) < 0.1), r_in
    assert np.all(np.abs(r_wall - 3) < 0.1), r_wall


def mean_abs_error(n, k, r, T):
    """The paper's mean absolute error over the time levels (the reading
    under which the C4 column of Table cfl is reproduced)."""
    h = 1.0 / n
    ht = r * h
    nt = int(round(T / ht))
    p = NCProblem(n, r)
    for name, v in mode_fields(2, n, k, 0.0, ht / 2, with_laplacian=False).items():
        p.set(name, v)
    tot = 0.0
    for s in range(1, nt + 1):
        p.step(1)
        ex = mode_fields(2, n, k, s * ht, (s + 0.5) * ht, with_laplacian=False)
        tot += sum(np.abs(p.get(a) - ex[a]).sum() for a in ("ez", "hx", "hy"))
    return tot / (3 * nt * n * n)


def test_table_cfl_nc_column():
    rows = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table_cfl_nc.txt"),
                      comments="#")
    for j, printed in rows:
        r = j / (6 * np.sqrt(2))
        got = mean_abs_error(64, (2, 2), r, 4 / np.sqrt(2))
        assert abs(got / printed - 1) < 0.03, (j, got, printed)


def test_table_cfl_nc_unstable_row():
    n, r = 64, 1 / np.sqrt(2)
    p = NCProblem(n, r)
    for name, v in mode_fields(2, n, (2, 2), 0.0, r / n / 2, with_laplacian=False).items():
        p.set(name, v)
    p.step(int(round((4 / np.sqrt(2)) / (r / n))))
    ez = p.get("ez")
    assert (not np.all(np.isfinite(ez))) or np.max(np.abs(ez)) > 1e3


def test_table_conv_rates_nc_column():
    r, T = 5 / (6 * np.sqrt(2)), 1 / np.sqrt(2)
    errs = {n: mean_abs_error(n, (2, 2), r, T) for n in (32, 64, 128)}
    assert abs(np.log2(errs[32] / errs[64]) - 1.98) < 0.05
    assert abs(np.log2(errs[64] / errs[128]) - 1.98) < 0.05
