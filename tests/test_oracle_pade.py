"""Pins of the oracle's staggered Pade derivative (Appendix A.1, eq:lhs).

* The printed closure rows and the interior rows are exact for quartic
  polynomials (their Taylor moments match through third order), so any wrong
  entry, sign or index in the assembled matrix breaks exactness.
* The banded elimination agrees with a dense solve of the printed matrix.
* Under the image closure the operator maps a sampled sine (cosine) mode to
  a cosine (sine) mode scaled by 2 sin(theta/2) / a(theta).
* Smooth non-polynomial data converge at fourth order for both closures.
"""
import numpy as np
import pytest

import oracle


def _points(n_in, node_to_half):
    """Input and output abscissae of one line with h = 1 / n."""
    if node_to_half:            # n_in = N+1 nodes -> N half points
        n = n_in - 1
        x_in = np.arange(n_in) / n
        x_out = (np.arange(n_in - 1) + 0.5) / n
    else:                       # n_in = N half points -> N-1 interior nodes
        n = n_in
        x_in = (np.arange(n_in) + 0.5) / n
        x_out = np.arange(1, n_in) / n
    return n, x_in, x_out


@pytest.mark.parametrize("node_to_half", [True, False])
@pytest.mark.parametrize("n_in", [5, 9, 17, 33])
def test_paper_closure_exact_on_quartics(node_to_half, n_in):
    rng = np.random.default_rng(7 + n_in)
    c = rng.normal(size=5)
    n, x_in, x_out = _points(n_in, node_to_half)
    f = np.polyval(c, x_in)
    fp = np.polyval(np.polyder(c), x_out)
    got = oracle.pade_line(f, oracle.CLOSURE_PAPER, node_to_half) * n
    assert np.max(np.abs(got - fp)) <= 1e-11 * (1 + np.max(np.abs(fp)))


def test_paper_closure_not_exact_for_quintics():
    # sanity of the pin above: degree 5 is no longer reproduced
    n, x_in, x_out = _points(17, True)
    f = x_in ** 5
    got = oracle.pade_line(f, oracle.CLOSURE_PAPER, True) * n
    assert np.max(np.abs(got - 5 * x_out ** 4)) > 1e-6


def _dense_printed(m, closure, node_to_half):
    a = np.zeros((m, m))
    for i in range(m):
        a[i, i] = 22.0
        if i > 0:
            a[i, i - 1] = 1.0
        if i < m - 1:
            a[i, i + 1] = 1.0
    if closure == oracle.CLOSURE_PAPER:
        a[0, :4] = [26.0, -5.0, 4.0, -1.0]
        a[m - 1, m - 4:] = [-1.0, 4.0, -5.0, 26.0]
    else:
        a[0, 0] = a[m - 1, m - 1] = 23.0 if node_to_half else 22.0
    return a / 24.0


@pytest.mark.parametrize("closure", [oracle.CLOSURE_PAPER, oracle.CLOSURE_REFLECT])
@pytest.mark.parametrize("node_to_half", [True, False])
def test_banded_solve_matches_dense(closure, node_to_half):
    rng = np.random.default_rng(11)
    f = rng.normal(size=41)
    d = np.diff(f)
    ref = np.linalg.solve(_dense_printed(d.size, closure, node_to_half), d)
    got = oracle.pade_line(f, closure, node_to_half)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [1, 3, 7, 15])
def test_reflect_symbol_on_modes(k):
    n = 32
    th = np.pi * k / n
    sym = 2 * np.sin(th / 2) / ((22 + 2 * np.cos(th)) / 24)
    # nodes -> half points: sin -> cos
    _, x_in, x_out = _points(n + 1, True)
    got = oracle.pade_line(np.sin(np.pi * k * x_in), oracle.CLOSURE_REFLECT, True)
    assert np.max(np.abs(got - sym * np.cos(np.pi * k * x_out))) < 1e-14
    # half points -> interior nodes: cos -> -sin
    _, x_in, x_out = _points(n, False)
    got = oracle.pade_line(np.cos(np.pi * k * x_in), oracle.CLOSURE_REFLECT, False)
    assert np.max(np.abs(got + sym * np.sin(np.pi * k * x_out))) < 1e-14


@pytest.mark.parametrize("closure", [oracle.CLOSURE_PAPER, oracle.CLOSURE_REFLECT])
@pytest.mark.parametrize("node_to_half", [True, False])
def test_fourth_order(closure, node_to_half):
    errs = []
    for n in (32, 64, 128, 256):
        n_in = n + 1 if node_to_half else n
        _, x_in, x_out = _points(n_in, node_to_half)
        # odd about the walls for nodes (sine-like), even for half points, so
        # that the image closure is consistent too
        if node_to_half:
            f, fp = np.sin(3 * np.pi * x_in), 3 * np.pi * np.cos(3 * np.pi * x_out)
        else:
            f, fp = np.cos(3 * np.pi * x_in), -3 * np.pi * np.sin(3 * np.pi * x_out)
        got = oracle.pade_line(f, closure, node_to_half) * n
        errs.append(np.max(np.abs(got - fp)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8), rates
