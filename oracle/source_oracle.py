"""One step of the 2D TM compact scheme with a current J = (0, 0, Jz):
Section 3.1 (eq:mh, Table tab:spec) with the ghost values of Section 3.3
(Method 2, eq:gst2).  TEST INFRASTRUCTURE ONLY.

It holds its own fields and calls the C oracle only for library-like steps:
the Pade derivative of one line (eq:lhs) and the CG solve of M with the
homogeneous wall rows.

Readings (the printed source terms disagree with the derivation that
precedes them; this follows the derivation):
  * Step 1 (E at t^{n+1/2}): phi = delta_t Ez solves -Delta phi + k^2 phi =
    k^2 F with k^2 = 24/h_t^2 and
        F = Z (curl H)_z + F_J,   F_J = -Z (Jz + (h_t^2/24) d^2Jz/dt^2)
    (the gradient of div J vanishes in the TM reduction).  The derivation
    gives d^3E/dt^3 = Z grad div J + Delta dE/dt - Z d^2J/dt^2, hence this
    F_J; the printed P(J) has the opposite signs on its last two terms and
    lacks 24/h_t^2 on J.
  * Step 2 (H at t^{n+1}): F = -(1/Z) curl E + (h_t^2/24) curl dJ/dt, from
    d^3H/dt^3 = Delta dH/dt + curl dJ/dt (the printed form carries
    -curl d^2J/dt^2).
  * The J part of F enters with its known Laplacian, the eq:helm2 form:
    scaled by h_t^2/24 it adds G_J = alpha F_J + h^2 Delta F_J / 12 to the
    right-hand side, with Delta F_J taken from the caller.
  * Ghosts along a half-point axis (eq:gst2): phi(-h/2) = phi(h/2) - h q_lo,
    phi(1 + h/2) = phi(1 - h/2) + h q_hi, q = phi_n + (h^2/24) phi_nnn from
    the caller's first and third normal derivatives at the wall.  Step 1
    uses them for H itself inside G(H) (the source conditioning, applied to
    H before its Pade curl); Step 2 uses them for delta_t H in the rows of
    M next to the walls, where the inhomogeneous part moves to the
    right-hand side.  Ez has no half-point axis: no ghosts.

Scaling as in the C oracle: M = alpha I - beta L9, Phi = h delta_t (field),
curl^A = h curl_h, so the J terms enter the right-hand side multiplied by h.
Arrays are (1, ny, nx) as everywhere in the oracle.
"""
from __future__ import annotations

import numpy as np

from .oracle import CLOSURE_PAPER, LAP_TRACKED, OracleProblem, pade_line


def _q(first, third, h):
    """eq:gst2: the ghost offset per unit h along a half-point axis."""
    return np.asarray(first, dtype=np.float64) + h * h / 24.0 * np.asarray(third, dtype=np.float64)


def _ext(a, half_x: bool, half_y: bool, qx=None, qy=None, h=1.0):
    """a (ny, nx) padded by one point on every side.  Along a half-point
    axis the ghosts follow eq:gst2 with offsets q (lo, hi), each an array
    along the other axis (node points 0..N); along a node axis the padding
    is never read and stays zero."""
    ny, nx = a.shape
    e = np.zeros((ny + 2, nx + 2))
    e[1:-1, 1:-1] = a
    if half_y:
        lo, hi = qy if qy is not None else (np.zeros(nx), np.zeros(nx))
        e[0, 1:-1] = a[0, :] - h * lo
        e[-1, 1:-1] = a[-1, :] + h * hi
    if half_x:
        lo, hi = qx if qx is not None else (np.zeros(ny), np.zeros(ny))
        e[1:-1, 0] = a[:, 0] - h * lo
        e[1:-1, -1] = a[:, -1] + h * hi
    return e


def _dxx(e):
    return e[1:-1, :-2] - 2.0 * e[1:-1, 1:-1] + e[1:-1, 2:]


def _dyy(e):
    return e[:-2, 1:-1] - 2.0 * e[1:-1, 1:-1] + e[2:, 1:-1]


def _dxxdyy(e):
    """D_xx D_yy on the interior of a padded array (the corner terms)."""
    c = e[:-2, :-2] + e[:-2, 2:] + e[2:, :-2] + e[2:, 2:]
    f = e[:-2, 1:-1] + e[2:, 1:-1] + e[1:-1, :-2] + e[1:-1, 2:]
    return c - 2.0 * f + 4.0 * e[1:-1, 1:-1]


def l9(e):
    """h^2 (Delta_h + h^2/6 Upsilon_h) in grid units (eq:ell, 2D)."""
    return _dxx(e) + _dyy(e) + _dxxdyy(e) / 6.0


class SourcedTM:
    """The 2D TM fields stepped with sources.  Ez and lz on (1, N+1, N+1),
    Hx on (1, N, N+1), Hy on (1, N+1, N)."""

    def __init__(self, n: int, r: float, z: float = 1.0, lap_mode: int = LAP_TRACKED):
        self.n, self.r, self.z, self.lap_mode = n, r, z, lap_mode
        self.h = 1.0 / n
        self.alpha = 1.0 + 2.0 / (r * r)
        self.beta = r * r / 24.0
        self.o = OracleProblem(2, n, r, z, closure=CLOSURE_PAPER, lap_mode=lap_mode)
        self.f = {}

    def close(self):
        self.o.close()

    def set(self, name, arr):
        self.f[name] = np.array(arr, dtype=np.float64).reshape(self.o.shape(name))

    def get(self, name):
        return self.f[name].copy()

    # -- Step 1 ------------------------------------------------------------
    def _g_h(self, d1):
        """G(H) = alpha H + h^2 Delta_h H / 12 with the eq:gst2 ghosts of H."""
        h, n = self.h, self.n
        hx, hy = self.f["hx"][0], self.f["hy"][0]
        qx = [_q(d1["hx_wall"][w][0], d1["hx_wall"][w][1], h) for w in (0, 1)]
        qy = [_q(d1["hy_wall"][w][0], d1["hy_wall"][w][1], h) for w in (0, 1)]
        ex = _ext(hx, half_x=False, half_y=True, qy=qx, h=h)
        ey = _ext(hy, half_x=True, half_y=False, qx=qy, h=h)
        gx = np.zeros_like(hx)
        gy = np.zeros_like(hy)
        # interior of the node axis only (x for Hx, y for Hy); the node walls
        # are never sources of a derivative at an Ez unknown
        gx[:, 1:n] = self.alpha * hx[:, 1:n] + (_dxx(ex) + _dyy(ex))[:, 1:n] / 12.0
        gy[1:n, :] = self.alpha * hy[1:n, :] + (_dxx(ey) + _dyy(ey))[1:n, :] / 12.0
        return gx, gy

    def _curl_e(self, hx, hy):
        """curl^A of (Hx, Hy) at the Ez unknowns: dHy/dx - dHx/dy (eq:lhs)."""
        n = self.n
        out = np.zeros((n + 1, n + 1))
        for j in range(1, n):
            out[j, 1:n] += pade_line(hy[j, :], CLOSURE_PAPER, False)
        for i in range(1, n):
            out[1:n, i] -= pade_line(hx[:, i], CLOSURE_PAPER, False)
        return out

    def half_step_e(self, d1):
        n, h, r, z = self.n, self.h, self.r, self.z
        ht2 = (r * h) ** 2 / 24.0
        fj = -z * (d1["jz"][0] + ht2 * d1["jz_tt"][0])                  # F_J
        lj = -z * h * h * (d1["jz_lap"][0] + ht2 * d1["jz_tt_lap"][0])   # h^2 Delta F_J
        gx, gy = self._g_h(d1)
        b = z * self._curl_e(gx, gy) + h * (self.alpha * fj + lj / 12.0)
        b[0, :] = b[-1, :] = 0.0
        b[:, 0] = b[:, -1] = 0.0
        phi = self.o.solve_m("ez", b[None])[0]
        e_old = self.f["ez"][0].copy()
        self.f["ez"][0, 1:n, 1:n] = e_old[1:n, 1:n] + r * phi[1:n, 1:n]
        if self.lap_mode == LAP_TRACKED:
            craw = z * self._curl_e(self.f["hx"][0], self.f["hy"][0]) + h * fj
            lz = self.f["lz"][0]
            lz[1:n, 1:n] += (24.0 / (r * r) * (self.f["ez"][0] - e_old) - 24.0 / r * craw)[1:n, 1:n]

    # -- Step 2 ------------------------------------------------------------
    def _g_e(self, d2):
        """alpha E + l/12 (carried l) or alpha E + h^2 Delta_h E / 12 at the
        interior nodes; on the walls, where Ez = 0, h^2 Delta Ez / 12 with
        Delta Ez = Z dJz/dt there (the wave equation with d^2Ez/dt^2 = 0)."""
        n, h = self.n, self.h
        e = self.f["ez"][0]
        g = h * h * self.z * d2["jz_t"][0] / 12.0
        g[1:n, 1:n] = 0.0
        if self.lap_mode == LAP_TRACKED:
            g[1:n, 1:n] = self.alpha * e[1:n, 1:n] + self.f["lz"][0][1:n, 1:n] / 12.0
        else:
            ee = _ext(e, False, False)
            g[1:n, 1:n] = (self.alpha * e + (_dxx(ee) + _dyy(ee)) / 12.0)[1:n, 1:n]
        return g

    def half_step_h(self, d2):
        n, h, r, z = self.n, self.h, self.r, self.z
        ht2 = (r * h) ** 2 / 24.0
        ge = self._g_e(d2)
        for name, half_x in (("hx", False), ("hy", True)):
            k = d2["kx" if name == "hx" else "ky"][0]
            kl = d2["kx_lap" if name == "hx" else "ky_lap"][0]
            fj = ht2 * k
            lj = h * h * ht2 * kl
            b = np.zeros_like(self.f[name][0])
            if name == "hx":     # -(1/Z) dEz/dy at (node x, half y)
                for i in range(1, n):
                    b[:, i] = -pade_line(ge[:, i], CLOSURE_PAPER, True) / z
                b[:, 1:n] += h * (self.alpha * fj + lj / 12.0)[:, 1:n]
            else:                # +(1/Z) dEz/dx at (half x, node y)
                for j in range(1, n):
                    b[j, :] = pade_line(ge[j, :], CLOSURE_PAPER, True) / z
                b[1:n, :] += h * (self.alpha * fj + lj / 12.0)[1:n, :]
            # M with the eq:gst2 ghosts of Phi = h delta_t H is affine:
            # M_inh(x) = M(x) + M_inh(0); the constant part moves to b
            wall = d2["dhx_wall"] if name == "hx" else d2["dhy_wall"]
            q = [h * _q(wall[w][0], wall[w][1], h) for w in (0, 1)]
            for w in (0, 1):           # Phi vanishes on the node walls, so do its ghosts
                q[w] = q[w].copy()
                q[w][0] = q[w][-1] = 0.0
            zero = np.zeros_like(b)
            ez = _ext(zero, half_x, not half_x, qx=q if half_x else None, qy=None if half_x else q, h=h)
            m0 = -self.beta * l9(ez)
            if half_x:
                b[1:n, :] -= m0[1:n, :]
            else:
                b[:, 1:n] -= m0[:, 1:n]
            phi = self.o.solve_m(name, b[None])[0]
            if half_x:
                self.f[name][0, 1:n, :] += r * phi[1:n, :]
            else:
                self.f[name][0, :, 1:n] += r * phi[:, 1:n]

    def step(self, d1, d2):
        self.half_step_e(d1)
        self.half_step_h(d2)
