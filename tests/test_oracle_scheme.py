"""Pins of the oracle's full time step (Section 3.4, Step 1 and Step 2).

* REFLECT closure: a single sampled cavity mode evolves by a closed-form
  amplitude recurrence (tests/closed_form.py), 2D and 3D, both ways of
  carrying the Laplacian of E, Z = 1 and Z != 1.
* PAPER closure: the printed errors of Table cfl (C4 column), the printed
  convergence rates of Table conv_rates (C4 column), blow-up at r = 1/sqrt(2)
  (Table cfl, last row; stability bound stabCFL).
* Structure: under REFLECT the Pade divergence of H (and of E in 3D) is
  conserved exactly for arbitrary data; the dense one-step map has spectral
  radius <= 1 below the CFL bound and > 1 above it (Section 4).
"""
import os

import numpy as np
import pytest

import closed_form as cf
import oracle
from workloads import field_shape, grid_coords, mode_fields, mode_omega, polarisation_3d

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def _start(p, dim, n, k, r, z=1.0, amp=1.0):
    h = 1.0 / n
    f = mode_fields(dim, n, k, 0.0, r * h / 2, amp=amp, z=z)
    for name, v in f.items():
        p.set(name, v)
    return f


@pytest.mark.parametrize("lap", [oracle.LAP_TRACKED, oracle.LAP_DISCRETE])
@pytest.mark.parametrize("n,k,r,z", [(16, (2, 3), 0.5, 1.0), (24, (5, 1), 0.589, 2.0), (12, (11, 11), 0.3, 0.5)])
def test_reflect_closed_form_2d(lap, n, k, r, z):
    h = 1.0 / n
    ns = 30
    p = oracle.OracleProblem(2, n, r, z, closure=oracle.CLOSURE_REFLECT, lap_mode=lap)
    _start(p, 2, n, k, r, z)
    p.step(ns)
    w = mode_omega(k)
    amps = (1.0, -np.pi * k[1] / (z * w) * np.sin(w * r * h / 2),
            np.pi * k[0] / (z * w) * np.sin(w * r * h / 2), -(h * np.pi) ** 2 * (k[0] ** 2 + k[1] ** 2))
    A, Bx, By, C = cf.evolve_2d(k, n, r, z, amps, ns, tracked=(lap == oracle.LAP_TRACKED))
    pats = {"ez": (A, np.sin, np.sin), "hx": (Bx, np.sin, np.cos), "hy": (By, np.cos, np.sin)}
    if lap == oracle.LAP_TRACKED:
        pats["lz"] = (C, np.sin, np.sin)
    for name, (amp, fx, fy) in pats.items():
        zc, yc, xc = grid_coords(name if name != "lz" else "ez", 2, n)
        ref = amp * fx(np.pi * k[0] * xc) * fy(np.pi * k[1] * yc)
        got = p.get(name)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), name


@pytest.mark.parametrize("lap", [oracle.LAP_TRACKED, oracle.LAP_DISCRETE])
def test_reflect_closed_form_3d(lap):
    n, k, r, z = 10, (2, 3, 4), 0.4, 1.0
    h = 1.0 / n
    ns = 12
    p = oracle.OracleProblem(3, n, r, z, closure=oracle.CLOSURE_REFLECT, lap_mode=lap)
    _start(p, 3, n, k, r, z)
    p.step(ns)
    kv = np.array(k, float)
    e = polarisation_3d(kv)
    w = mode_omega(k)
    b0 = -np.pi / (z * w) * np.cross(kv, e) * np.sin(w * r * h / 2)
    c0 = -(h * np.pi) ** 2 * (kv @ kv) * e
    a, b, c = cf.evolve_3d(k, n, r, z, e, b0, c0, ns, tracked=(lap == oracle.LAP_TRACKED))
    for s, ax in enumerate("xyz"):
        for kind, amp in (("e", a[s]), ("h", b[s])):
            name = kind + ax
            zc, yc, xc = grid_coords(name, 3, n)
            fn = [np.sin, np.sin, np.sin] if kind == "e" else [np.cos, np.cos, np.cos]
            fn[s] = np.cos if kind == "e" else np.sin
            ref = amp * fn[0](np.pi * k[0] * xc) * fn[1](np.pi * k[1] * yc) * fn[2](np.pi * k[2] * zc)
            got = p.get(name)
            assert np.linalg.norm(got - ref) <= 1e-12 * max(np.linalg.norm(ref), 1e-300), name


def mean_abs_error(n, k, r, T, closure=oracle.CLOSURE_PAPER, lap=oracle.LAP_TRACKED):
    """The mean absolute error of Section 5.1, summed over the time levels
    n = 1..N_tau and all stored points, divided by 3 N_tau N^2; E at n h_tau,
    H at (n + 1/2) h_tau; N_tau = round(T / h_tau)."""
    h = 1.0 / n
    ht = r * h
    nt = int(round(T / ht))
    p = oracle.OracleProblem(2, n, r, 1.0, closure=closure, lap_mode=lap)
    _start(p, 2, n, k, r)
    tot = 0.0
    for s in range(1, nt + 1):
        p.step(1)
        ex = mode_fields(2, n, k, s * ht, (s + 0.5) * ht, with_laplacian=False)
        for name in ("ez", "hx", "hy"):
            tot += np.abs(p.get(name) - ex[name]).sum()
    return tot / (3 * nt * n * n)


def test_table_cfl_c4_column():
    rows = _load("table_cfl_c4.txt")
    for j, printed in rows:
        r = j / (6 * np.sqrt(2))
        got = mean_abs_error(64, (2, 2), r, 4 / np.sqrt(2))
        # the reading of the error metric is the paper's only loose end; the
        # scheme itself reproduces the printed values to about 2 %
        assert abs(got / printed - 1) < 0.03, (j, got, printed)


def test_table_cfl_unstable_row():
    # r = 1/sqrt(2) exceeds the stability bound (stabCFL); Table cfl prints inf
    n = 64
    r = 1 / np.sqrt(2)
    p = oracle.OracleProblem(2, n, r, 1.0)
    _start(p, 2, n, (2, 2), r)
    h = 1.0 / n
    p.step(int(round((4 / np.sqrt(2)) / (r * h))))
    ez = p.get("ez")
    assert (not np.all(np.isfinite(ez))) or np.max(np.abs(ez)) > 1e3


def test_table_conv_rates_c4_column():
    rows = _load("table_conv_rates_c4.txt")
    cache = {}
    for j, n, printed in rows:
        r = j / (6 * np.sqrt(2))
        for m in (int(n) // 2, int(n)):
            if (j, m) not in cache:
                cache[(j, m)] = mean_abs_error(m, (2, 2), r, 1 / np.sqrt(2))
        rate = np.log2(cache[(j, int(n) // 2)] / cache[(j, int(n))])
        assert abs(rate - printed) < 0.15, (j, n, rate, printed)


def _pade_div_2d(hx, hy, n, closure):
    """delta_x Hx + delta_y Hy at the cell centres (x_{i+1/2}, y_{j+1/2})."""
    hx = hx[0]
    hy = hy[0]
    dx = np.stack([oracle.pade_line(hx[j], closure, True) for j in range(n)])          # (N, N)
    dy = np.stack([oracle.pade_line(hy[:, i], closure, True) for i in range(n)]).T     # (N, N)
    return dx + dy


def _random_state(p, dim, n, rng):
    for name in p.fields():
        p.set(name, rng.normal(size=p.shape(name)))
    # H normal to a wall is constant in time; start it at zero
    for name in (["hx", "hy"] if dim == 2 else ["hx", "hy", "hz"]):
        a = p.get(name)
        ax = "xyz".index(name[1])
        sl = [slice(None)] * 3
        sl[2 - ax] = 0
        a[tuple(sl)] = 0
        sl[2 - ax] = -1
        a[tuple(sl)] = 0
        p.set(name, a)


@pytest.mark.parametrize("lap", [oracle.LAP_TRACKED, oracle.LAP_DISCRETE])
def test_reflect_conserves_pade_divergence_2d(lap):
    n = 16
    rng = np.random.default_rng(3)
    p = oracle.OracleProblem(2, n, 0.5, 1.0, closure=oracle.CLOSURE_REFLECT, lap_mode=lap)
    _random_state(p, 2, n, rng)
    d0 = _pade_div_2d(p.get("hx"), p.get("hy"), n, oracle.CLOSURE_REFLECT)
    p.step(20)
    d1 = _pade_div_2d(p.get("hx"), p.get("hy"), n, oracle.CLOSURE_REFLECT)
    assert np.max(np.abs(d1 - d0)) < 1e-12 * np.max(np.abs(d0))


def _pade_div_3d(p, kind, n, closure):
    """Pade divergence of E (at nodes) or H (at cell centres) in 3D."""
    tot = 0
    for s, ax in enumerate("xyz"):
        a = p.get(kind + ax)
        axis = 2 - s
        out = np.apply_along_axis(lambda v: oracle.pade_line(v, closure, kind == "h"), axis, a)
        # restrict the other axes to the common grid of the divergence
        sl = [slice(None)] * 3
        for t in range(3):
            if t != s and kind == "e":
                sl[2 - t] = slice(1, n)         # interior nodes
        tot = tot + out[tuple(sl)]
    return tot


def test_reflect_conserves_pade_divergence_3d():
    n = 8
    rng = np.random.default_rng(4)
    p = oracle.OracleProblem(3, n, 0.4, 1.0, closure=oracle.CLOSURE_REFLECT)
    _random_state(p, 3, n, rng)
    dh0, de0 = _pade_div_3d(p, "h", n, 1), _pade_div_3d(p, "e", n, 1)
    p.step(6)
    dh1, de1 = _pade_div_3d(p, "h", n, 1), _pade_div_3d(p, "e", n, 1)
    assert np.max(np.abs(dh1 - dh0)) < 1e-12 * np.max(np.abs(dh0))
    assert np.max(np.abs(de1 - de0)) < 1e-12 * np.max(np.abs(de0))


def _one_step_matrix(n, r, closure, lap):
    p = oracle.OracleProblem(2, n, r, 1.0, closure=closure, lap_mode=lap)
    names = ["ez", "hx", "hy"] + (["lz"] if lap == oracle.LAP_TRACKED else [])
    sizes = [int(np.prod(p.shape(a))) for a in names]
    tot = sum(sizes)
    mat = np.zeros((tot, tot))
    for col in range(tot):
        v = np.zeros(tot)
        v[col] = 1.0
        off = 0
        for a, s in zip(names, sizes):
            p.set(a, v[off:off + s])
            off += s
        p.step(1)
        mat[:, col] = np.concatenate([p.get(a).ravel() for a in names])
    return mat


@pytest.mark.parametrize("closure", [oracle.CLOSURE_PAPER, oracle.CLOSURE_REFLECT])
def test_one_step_spectral_radius(closure):
    n = 16
    for r, stable in ((0.5, True), (5 / (6 * np.sqrt(2)), True), (1 / np.sqrt(2), False)):
        rho = np.max(np.abs(np.linalg.eigvals(_one_step_matrix(n, r, closure, oracle.LAP_DISCRETE))))
        if stable:
            assert rho <= 1 + 1e-10, (r, rho)
        else:
            assert rho > 1.05, (r, rho)
    # carried Laplacian: eigenvalue one may be defective but nothing grows
    rho = np.max(np.abs(np.linalg.eigvals(_one_step_matrix(n, 0.5, closure, oracle.LAP_TRACKED))))
    assert rho <= 1 + 1e-6, rho


def test_paper_closure_converges_at_fourth_order_l2():
    # relative L2 over all fields at T = 1 for mode (4, 3), CFL 0.5
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        r = 0.5
        nt = int(round(1.0 / (r * h)))
        p = oracle.OracleProblem(2, n, r)
        _start(p, 2, n, (4, 3), r)
        p.step(nt)
        ex = mode_fields(2, n, (4, 3), nt * r * h, (nt + 0.5) * r * h, with_laplacian=False)
        num = sum(np.sum((p.get(a) - ex[a]) ** 2) for a in ("ez", "hx", "hy"))
        den = sum(np.sum(ex[a] ** 2) for a in ("ez", "hx", "hy"))
        errs.append(np.sqrt(num / den))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.3), (errs, rates)


@pytest.mark.parametrize("lap", [oracle.LAP_TRACKED, oracle.LAP_DISCRETE])
def test_paper_closure_converges_3d(lap):
    """The 3D PAPER path (no 3D numbers in the paper): relative L2 over all
    six fields against the exact cube-cavity mode (1, 2, 1), CFL 0.4,
    T = 0.5, falls at least at fourth order (observed about 5 on these
    grids, as the PAPER rows give in 2D)."""
    k = (1, 2, 1)
    names = ["ex", "ey", "ez", "hx", "hy", "hz"]
    ns = (12, 24, 36)
    errs = []
    for n in ns:
        h, r = 1.0 / n, 0.4
        nt = int(round(0.5 / (r * h)))
        p = oracle.OracleProblem(3, n, r, lap_mode=lap)
        _start(p, 3, n, k, r)
        p.step(nt)
        ex = mode_fields(3, n, k, nt * r * h, (nt + 0.5) * r * h, with_laplacian=False)
        num = sum(np.sum((p.get(a) - ex[a]) ** 2) for a in names)
        den = sum(np.sum(ex[a] ** 2) for a in names)
        errs.append(np.sqrt(num / den))
        p.close()
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    assert min(rates) > 3.8, (errs, rates)
