"""Pins of the oracle's right-hand sides and of its signed half-steps.

* oc_rhs: the right-hand side of each elliptic system (Section 3.4: Step 1
  Z curl^A G(H), Step 2 -(1/Z) curl^A G_E) equals a dense assembly written
  here from the definitions alone: the source conditioning G u = alpha u +
  (second differences)/12 with the even ghost along half-point axes and the
  wall values along node axes (Corollary cor:ghost_cor, Table tab:bc), the
  conditioned E source alpha E + l/12 (or alpha E + L5 E/12) vanishing on
  E's walls, and the staggered Pade derivative A^{-1} D as a dense solve
  with the printed rows of eq:lhs.  2D and 3D, both closures, both ways of
  carrying the Laplacian, random data with non-zero normal H on the walls.
* Time reversibility: the staggered update E += r Phi_E(H), H += r Phi_H(E)
  (with the carried Laplacian l += (24/r^2) dE - (24/r) Z curl^A H) is
  undone exactly by the same half-steps with -r in reverse order, so n
  steps forward and n backward return the start to rounding.
"""
import numpy as np
import pytest

import oracle
from gpu_util import random_fields
from workloads import component_half_axes, component_names, field_shape

AX = "xyz"


def _pade_dense(n_in, closure, node_to_half):
    """A^{-1} D for one line (no 1/h), from the printed rows of eq:lhs."""
    m = n_in - 1
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
    d = np.zeros((m, n_in))
    for i in range(m):
        d[i, i], d[i, i + 1] = -1.0, 1.0
    return np.linalg.solve(a / 24.0, d)


def _cond(u, name, dim, alpha):
    """alpha u + (sum of second differences)/12; even ghost along half axes,
    stored wall values along node axes (zero padding beyond, only reached
    at wall points, which no line of a curl uses as a G(H) value)."""
    half = component_half_axes(name, dim)
    lap = np.zeros_like(u)
    for a in range(dim):
        ax = 2 - a
        pad = [(0, 0)] * 3
        pad[ax] = (1, 1)
        up = np.pad(u, pad, mode="edge" if half[a] else "constant")
        sl_m = [slice(None)] * 3
        sl_p = [slice(None)] * 3
        sl_m[ax] = slice(0, -2)
        sl_p[ax] = slice(2, None)
        lap += up[tuple(sl_m)] + up[tuple(sl_p)] - 2 * u
    return alpha * u + lap / 12.0


def _zero_node_walls(name, dim, a):
    half = component_half_axes(name, dim)
    a = a.copy()
    for ax in range(dim):
        if not half[ax]:
            sl = [slice(None)] * 3
            for idx in (0, -1):
                sl[2 - ax] = idx
                a[tuple(sl)] = 0.0
    return a


def _deriv(src, name_src, dim, axis, closure):
    """Pade derivative of the array src along `axis` (x = 0)."""
    half = component_half_axes(name_src, dim)
    ax = 2 - axis
    op = _pade_dense(src.shape[ax], closure, node_to_half=not half[axis])
    return np.moveaxis(np.tensordot(op, np.moveaxis(src, ax, 0), axes=(1, 0)), 0, ax)


def _place(der, name_tgt, dim, n, axis):
    """Put the n_out derivative values along `axis` onto the target grid."""
    out = np.zeros(field_shape(name_tgt, dim, n))
    half = component_half_axes(name_tgt, dim)
    sl = [slice(None)] * 3
    sl[2 - axis] = slice(0, n) if half[axis] else slice(1, n)
    out[tuple(sl)] = der
    return out


def _unknowns(name, dim, n):
    half = component_half_axes(name, dim)
    sl = []
    for a in (2, 1, 0):
        sl.append(slice(0, 1) if a >= dim else (slice(0, n) if half[a] else slice(1, n)))
    return tuple(sl)


def _dense_rhs(f, tgt, dim, n, r, z, closure, lap_mode):
    alpha = 1 + 2 / r ** 2
    s = AX.index(tgt[1])
    s1, s2 = (s + 1) % 3, (s + 2) % 3
    if tgt[0] == "e":
        kind, scale = "h", z
    else:
        kind, scale = "e", -1.0 / z
    names = set(component_names(dim))

    def source(c):
        nm = kind + AX[c]
        if nm not in names:
            return None, nm
        if kind == "h":
            return _cond(f[nm], nm, dim, alpha), nm
        if lap_mode == oracle.LAP_TRACKED:
            g = alpha * f[nm] + f["l" + AX[c]] / 12.0
        else:
            g = _cond(f[nm], nm, dim, alpha)
        return _zero_node_walls(nm, dim, g), nm

    out = np.zeros(field_shape(tgt, dim, n))
    for axis, comp, sign in ((s1, s2, 1.0), (s2, s1, -1.0)):
        if axis >= dim:
            continue
        src, nm = source(comp)
        if src is None:
            continue
        out += sign * _place(_deriv(src, nm, dim, axis, closure), tgt, dim, n, axis)
    return scale * out


@pytest.mark.parametrize("closure", [oracle.CLOSURE_PAPER, oracle.CLOSURE_REFLECT])
@pytest.mark.parametrize("lap_mode", [oracle.LAP_TRACKED, oracle.LAP_DISCRETE])
@pytest.mark.parametrize("dim,n,r,z", [(2, 9, 0.5, 1.0), (2, 12, 0.45, 1.7), (3, 8, 0.4, 0.8)])
def test_rhs_matches_dense_assembly(closure, lap_mode, dim, n, r, z):
    f = random_fields(dim, n, seed=dim * 1000 + n, h_walls=True)
    p = oracle.OracleProblem(dim, n, r, z, closure=closure, lap_mode=lap_mode)
    for name, v in f.items():
        p.set(name, v)
    for tgt in component_names(dim):
        ref = _dense_rhs(f, tgt, dim, n, r, z, closure, lap_mode)
        got = p.rhs(tgt)
        sl = _unknowns(tgt, dim, n)
        assert np.max(np.abs(got[sl] - ref[sl])) <= 1e-12 * np.max(np.abs(ref[sl])), tgt


def test_dense_rhs_sees_normal_h_walls():
    # the pin above exercises the wall values: changing the normal H on a
    # wall changes the Step 1 right-hand side next to it
    dim, n, r = 2, 10, 0.5
    f = random_fields(dim, n, seed=4, h_walls=True)
    p = oracle.OracleProblem(dim, n, r)
    for name, v in f.items():
        p.set(name, v)
    before = p.rhs("ez")
    # the x = 0 wall of Hx, varying along the wall (a constant there has
    # zero y-derivative)
    f["hx"][:, :, 0] += np.linspace(0.0, 1.0, f["hx"].shape[1]) ** 2
    p.set("hx", f["hx"])
    after = p.rhs("ez")
    assert np.max(np.abs(after[:, 1:n, 1] - before[:, 1:n, 1])) > 1e-3


@pytest.mark.parametrize("closure", [oracle.CLOSURE_PAPER, oracle.CLOSURE_REFLECT])
@pytest.mark.parametrize("lap_mode", [oracle.LAP_TRACKED, oracle.LAP_DISCRETE])
@pytest.mark.parametrize("dim,n,r", [(2, 16, 0.5), (3, 8, 0.4)])
def test_time_reversibility(closure, lap_mode, dim, n, r):
    f = random_fields(dim, n, seed=77 + n)
    p = oracle.OracleProblem(dim, n, r, 1.3, closure=closure, lap_mode=lap_mode)
    for name, v in f.items():
        p.set(name, v)
    start = {a: p.get(a) for a in p.fields()}
    steps = 12
    p.step(steps)
    moved = {a: p.get(a) for a in p.fields()}
    for _ in range(steps):
        p.half_step_h(-r)
        p.half_step_e(-r)
    names = [a for a in p.fields() if a[0] in "eh"]
    if lap_mode == oracle.LAP_TRACKED:
        names += [a for a in p.fields() if a[0] == "l"]
    for a in names:
        back = p.get(a)
        scale = np.max(np.abs(start[a]))
        assert np.max(np.abs(back - start[a])) <= 1e-11 * scale, a
        # and the forward run did move the state
        assert np.max(np.abs(moved[a] - start[a])) > 1e-3 * scale, a
