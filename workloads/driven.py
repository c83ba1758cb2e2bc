"""A driven 2D TM cavity: a smooth exact solution of Maxwell's equations
with a current J = (0, 0, Jz) in the PEC unit square, for problems with
sources (Section 3.1).

    Ez = s(t) phi(x) psi(y),            s(t) = cos(w t),  S(t) = sin(w t)/w,
    Hx = -(1/Z) S(t) phi(x) psi'(y),    Hy = (1/Z) S(t) phi'(x) psi(y),
    Jz = dHy/dx - dHx/dy - (1/Z) dEz/dt,

with phi(x) = sin(pi x) e^{a x}, psi(y) = sin(pi y) e^{b y}.  Faraday's law
holds exactly, div H = 0, Ez vanishes on every wall and the normal H
components vanish on theirs; the Neumann data of the tangential H
components (dHx/dy at y = 0, 1 and dHy/dx at x = 0, 1) are not zero, since
psi''(0) = 2 pi b and phi''(0) = 2 pi a.

This module only samples the solution, the current and their derivatives on
the staggered grids; it holds no arithmetic of the scheme.  Every k-th
derivative of sin(pi x) e^{c x} is Im((c + i pi)^k e^{(c + i pi) x}).
"""
from __future__ import annotations

import numpy as np

from .cavity import grid_coords


def _deriv(c: float, k: int, x):
    q = complex(c, np.pi)
    return np.imag(q ** k * np.exp(q * x))


class DrivenTM:
    def __init__(self, z: float = 1.0, w: float = 2.0 * np.pi * 1.3, a: float = 0.7, b: float = -0.4):
        self.z, self.w, self.a, self.b = float(z), float(w), float(a), float(b)

    # time factors: s and S = int s, with their derivatives
    def _s(self, k: int, t: float) -> float:
        """k-th derivative of s(t) = cos(w t); k = -1 gives S(t) = sin(w t)/w."""
        w = self.w
        if k == -1:
            return np.sin(w * t) / w
        return w ** k * np.cos(w * t + k * np.pi / 2.0)

    def _pp(self, i: int, j: int, name: str, n: int):
        """phi^(i)(x) psi^(j)(y) on the grid of component `name`."""
        _, yc, xc = grid_coords(name, 2, n)
        return _deriv(self.a, i, xc) * _deriv(self.b, j, yc)

    def _jz_space(self, kt: int, t: float, n: int, name: str, lap: bool):
        """d^kt Jz / dt^kt on the grid of `name` (its Laplacian if lap):
        Jz = (1/Z) (S(t) (phi'' psi + phi psi'') - s'(t) phi psi)."""
        st = self._s(kt - 1, t)
        sd = self._s(kt + 1, t)
        if lap:
            a = self._pp(4, 0, name, n) + 2 * self._pp(2, 2, name, n) + self._pp(0, 4, name, n)
            bb = self._pp(2, 0, name, n) + self._pp(0, 2, name, n)
        else:
            a = self._pp(2, 0, name, n) + self._pp(0, 2, name, n)
            bb = self._pp(0, 0, name, n)
        return (st * a - sd * bb) / self.z

    def fields(self, n: int, tau_e: float, tau_h: float):
        """Ez and the carried Laplacian lz = h^2 Delta Ez at tau_e; Hx, Hy at tau_h."""
        h = 1.0 / n
        s_e, S_h = self._s(0, tau_e), self._s(-1, tau_h)
        out = {
            "ez": s_e * self._pp(0, 0, "ez", n),
            "hx": -S_h / self.z * self._pp(0, 1, "hx", n),
            "hy": S_h / self.z * self._pp(1, 0, "hy", n),
            "lz": h * h * s_e * (self._pp(2, 0, "ez", n) + self._pp(0, 2, "ez", n)),
        }
        for k in ("ez", "lz"):   # exact zeros on the Ez walls
            a = out[k]
            a[:, 0, :] = a[:, -1, :] = 0.0
            a[:, :, 0] = a[:, :, -1] = 0.0
        return {k: np.ascontiguousarray(v) for k, v in out.items()}

    def _walls(self, n: int, t: float, kt: int):
        """d^kt/dt^kt of the wall data: dHx/dy, d^3Hx/dy^3 at y = 0, 1 (along
        x = i h, i = 0..N) and dHy/dx, d^3Hy/dx^3 at x = 0, 1 (along y = j h)."""
        St = self._s(kt - 1, t) / self.z
        xs = np.arange(n + 1) / n
        hx = [[-St * _deriv(self.a, 0, xs) * _deriv(self.b, 1 + d, yw) for d in (1, 3)] for yw in (0.0, 1.0)]
        hy = [[St * _deriv(self.a, 1 + d, xw) * _deriv(self.b, 0, xs) for d in (1, 3)] for xw in (0.0, 1.0)]
        return hx, hy

    def step1_data(self, n: int, t: float):
        """Data of the E half-step at t = t^{n+1/2}: Jz, d^2Jz/dt^2 and their
        Laplacians on the Ez grid, the H wall data at t."""
        d = {
            "jz": self._jz_space(0, t, n, "ez", False),
            "jz_tt": self._jz_space(2, t, n, "ez", False),
            "jz_lap": self._jz_space(0, t, n, "ez", True),
            "jz_tt_lap": self._jz_space(2, t, n, "ez", True),
        }
        d["hx_wall"], d["hy_wall"] = self._walls(n, t, 0)
        return d

    def step2_data(self, n: int, t: float):
        """Data of the H half-step at t = t^{n+1}: dJz/dt on the Ez grid, K =
        curl dJ/dt on the Hx and Hy grids (Kx = d/dy dJz/dt, Ky = -d/dx
        dJz/dt) with their Laplacians, and the dH/dt wall data at t."""
        z = self.z
        s1 = self._s(0, t)        # S'
        s2 = self._s(2, t)        # s''

        def k_of(name, ix, iy, lap):
            if lap:
                a = (self._pp(4 + ix, iy, name, n) + 2 * self._pp(2 + ix, 2 + iy, name, n)
                     + self._pp(ix, 4 + iy, name, n))
                bb = self._pp(2 + ix, iy, name, n) + self._pp(ix, 2 + iy, name, n)
            else:
                a = self._pp(2 + ix, iy, name, n) + self._pp(ix, 2 + iy, name, n)
                bb = self._pp(ix, iy, name, n)
            return (s1 * a - s2 * bb) / z

        d = {
            "jz_t": self._jz_space(1, t, n, "ez", False),
            "kx": k_of("hx", 0, 1, False),
            "kx_lap": k_of("hx", 0, 1, True),
            "ky": -k_of("hy", 1, 0, False),
            "ky_lap": -k_of("hy", 1, 0, True),
        }
        d["dhx_wall"], d["dhy_wall"] = self._walls(n, t, 1)
        return d
