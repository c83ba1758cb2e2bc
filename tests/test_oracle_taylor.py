"""Pins of the oracle's Taylor start of H (Section 5.1, eq:talorh, J = 0):
H(h_tau/2) = H + a H_t + a^2/2 H_tt + a^3/6 H_ttt + a^4/24 H_tttt, a = h_tau/2,
with H_t = -(1/Z) curl E (Pade curl), H_tt = Delta_h H, H_ttt = Delta_h H_t,
H_tttt = Delta_h H_tt.

* REFLECT closure: every operator is diagonal on a sampled cavity mode, so
  H(h_tau/2) is a closed form: the Pade derivative maps sin to cos (and cos
  to -sin) with the factor s = 2 sin(theta/2) / a(theta), a = (22 + 2 cos
  theta)/24, and h^2 Delta_h multiplies by -sigma, sigma = sum 4 sin^2(theta/2)
  (2D and 3D, E only and H only, Z != 1).
* Accuracy: H(h_tau/2) against the exact mode converges at fourth order (both
  closures), and the compact scheme started from it ends within 3 % of the
  run started from the exact H(h_tau/2).
"""
import numpy as np
import pytest

import oracle
from workloads import grid_coords, mode_fields, polarisation_3d

AX = "xyz"


def _s(k, n):
    th = np.pi * k / n
    return 2 * np.sin(th / 2) / ((22 + 2 * np.cos(th)) / 24)


def _sig(k, n):
    return 4 * np.sin(np.pi * k / n / 2) ** 2


def _pattern(name, k, dim, n, funcs):
    zc, yc, xc = grid_coords(name, dim, n)
    coords = (xc, yc, zc)
    out = np.ones(np.broadcast_shapes(xc.shape, yc.shape, zc.shape))
    for a in range(dim):
        out = out * funcs[a](np.pi * k[a] * coords[a])
    return out


@pytest.mark.parametrize("n,k,r,z", [(16, (2, 3), 0.5, 1.0), (24, (5, 1), 0.4, 2.0), (12, (11, 7), 0.3, 0.7)])
def test_reflect_closed_form_2d_from_e(n, k, r, z):
    p = oracle.OracleProblem(2, n, r, z, closure=oracle.CLOSURE_REFLECT)
    f = mode_fields(2, n, k, 0.0, 0.0, z=z)                 # H(0) = 0 for the cavity mode
    for name, v in f.items():
        p.set(name, v)
    p.init_h_taylor()
    sig = _sig(k[0], n) + _sig(k[1], n)
    g = (r / 2 - r ** 3 * sig / 48) / z
    ref_hx = -g * _s(k[1], n) * _pattern("hx", k, 2, n, (np.sin, np.cos))
    ref_hy = g * _s(k[0], n) * _pattern("hy", k, 2, n, (np.cos, np.sin))
    for name, ref in (("hx", ref_hx), ("hy", ref_hy)):
        got = p.get(name)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), name


def test_reflect_closed_form_2d_from_h():
    # E = 0, H(0) a mode: H(h_tau/2) = (1 - r^2 sigma/8 + r^4 sigma^2/384) H(0)
    n, k, r = 20, (3, 4), 0.5
    p = oracle.OracleProblem(2, n, r, 1.0, closure=oracle.CLOSURE_REFLECT)
    f = mode_fields(2, n, k, 0.0, 0.3)
    f["ez"][:] = 0.0
    f["lz"][:] = 0.0
    for name, v in f.items():
        p.set(name, v)
    p.init_h_taylor()
    sig = _sig(k[0], n) + _sig(k[1], n)
    fac = 1 - r ** 2 * sig / 8 + r ** 4 * sig ** 2 / 384
    for name in ("hx", "hy"):
        assert np.max(np.abs(p.get(name) - fac * f[name])) <= 1e-13 * np.max(np.abs(f[name])), name


def test_reflect_closed_form_3d():
    n, k, r, z = 10, (2, 3, 4), 0.4, 1.3
    p = oracle.OracleProblem(3, n, r, z, closure=oracle.CLOSURE_REFLECT)
    f = mode_fields(3, n, k, 0.0, 0.0, z=z)
    for name, v in f.items():
        p.set(name, v)
    p.init_h_taylor()
    e = polarisation_3d(k)
    s = [_s(k[a], n) for a in range(3)]
    sig = sum(_sig(k[a], n) for a in range(3))
    g = (r / 2 - r ** 3 * sig / 48) / z
    for c in range(3):
        c1, c2 = (c + 1) % 3, (c + 2) % 3
        # (curl^A E)_c = delta_{c1} E_{c2} - delta_{c2} E_{c1}; every Pade
        # derivative of E turns its sine along that axis into a cosine
        amp = s[c1] * e[c2] - s[c2] * e[c1]
        funcs = [np.cos, np.cos, np.cos]
        funcs[c] = np.sin
        ref = -g * amp * _pattern("h" + AX[c], k, 3, n, funcs)
        got = p.get("h" + AX[c])
        assert np.max(np.abs(got - ref)) <= 1e-13 * (np.max(np.abs(ref)) + 1e-300), c


def _rel(a, b, names):
    return np.sqrt(sum(np.sum((a[x] - b[x]) ** 2) for x in names) / sum(np.sum(b[x] ** 2) for x in names))


@pytest.mark.parametrize("closure", [oracle.CLOSURE_PAPER, oracle.CLOSURE_REFLECT])
def test_taylor_start_is_fourth_order(closure):
    errs = []
    for n in (32, 64, 128):
        r = 0.5
        p = oracle.OracleProblem(2, n, r, 1.0, closure=closure)
        for name, v in mode_fields(2, n, (4, 3), 0.0, 0.0).items():
            p.set(name, v)
        p.init_h_taylor()
        ex = mode_fields(2, n, (4, 3), 0.0, r / n / 2)
        errs.append(_rel({a: p.get(a) for a in ("hx", "hy")}, ex, ("hx", "hy")))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.9), rates


def test_scheme_from_taylor_start_matches_exact_start():
    n, r = 64, 0.5
    ht = r / n
    steps = int(round(1 / ht))
    out = {}
    for start in ("taylor", "exact"):
        p = oracle.OracleProblem(2, n, r, 1.0)
        f = mode_fields(2, n, (4, 3), 0.0, ht / 2)
        if start == "taylor":
            f["hx"][:] = 0.0
            f["hy"][:] = 0.0
        for name, v in f.items():
            p.set(name, v)
        if start == "taylor":
            p.init_h_taylor()
        p.step(steps)
        ex = mode_fields(2, n, (4, 3), steps * ht, (steps + 0.5) * ht)
        out[start] = _rel({a: p.get(a) for a in ("ez", "hx", "hy")}, ex, ("ez", "hx", "hy"))
    assert abs(out["taylor"] / out["exact"] - 1) < 0.03, out
