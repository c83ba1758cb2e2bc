"""Plain FP64 CPU reference of the non-compact comparison scheme NC.

TEST INFRASTRUCTURE ONLY: the product package never imports this module.

NC (Section 5.2, "Comparable schemes") is the Yee update of the 2D TM
system (maxwell2d) with the first derivatives of stencil K4 at a = 0
(eq:K4): on the staggered line
    D u(x_i) = [ (9/8)(u(i+1/2) - u(i-1/2)) - (1/24)(u(i+3/2) - u(i-3/2)) ] / h,
i.e. c = (9 - 16a)/8 and d = (16a - 1)/24 at a = 0, and next to a wall,
where u(i-3/2) or u(i+3/2) falls outside the grid, the standard one-sided
approximation on the four nearest values (the paper names it, it does not
print it; this reading reproduces the NC column of Table cfl to 2 %),
    D u(x_i) = [ -23 u(i-1/2) + 21 u(i+1/2) + 3 u(i+3/2) - u(i+5/2) ] / (24 h)
(mirrored at the other wall): exact on cubics, third-order local
truncation error, fourth-order accuracy of the scheme in space.  Time stepping (the Yee updating rules of
Section 5.2):
    Ez^{n+1}   = Ez^n   + h_tau Z (Dx Hy^{n+1/2} - Dy Hx^{n+1/2})   (interior nodes)
    Hx^{n+3/2} = Hx^{n+1/2} - (h_tau / Z) Dy Ez^{n+1}
    Hy^{n+3/2} = Hy^{n+1/2} + (h_tau / Z) Dx Ez^{n+1}
Tangential Ez stays 0 on the walls; the normal H components keep their wall
values (maxwell2d with the PEC conditions of Section 2).  The impedance Z
enters as in maxwell2d.

Arrays are (1, ny, nx), x fastest, walls included, as everywhere else.
"""
from __future__ import annotations

import numpy as np

_INTERIOR = (1.0 / 24.0, -9.0 / 8.0, 9.0 / 8.0, -1.0 / 24.0)   # u(i-3/2), u(i-1/2), u(i+1/2), u(i+3/2)
_ONE_SIDED = (-23.0 / 24.0, 21.0 / 24.0, 3.0 / 24.0, -1.0 / 24.0)   # u(i-1/2), u(i+1/2), u(i+3/2), u(i+5/2)


def staggered_derivative(u: np.ndarray, n_out: int) -> np.ndarray:
    """D u along the last axis at the n_out output points, output k sitting
    midway between inputs k and k + 1 (h = 1; divide by h).

    Inputs u[..., 0 .. m-1] sit at half-integer positions relative to the
    outputs; every output uses the K4 row where its four neighbours exist
    and the one-sided row otherwise."""
    m = u.shape[-1]
    out = np.zeros(u.shape[:-1] + (n_out,))
    for k in range(n_out):
        left = k                               # input just left of output k
        if left - 1 >= 0 and left + 2 <= m - 1:
            idx, w = (left - 1, left, left + 1, left + 2), _INTERIOR
        elif left - 1 < 0:
            idx, w = (left, left + 1, left + 2, left + 3), _ONE_SIDED
        else:
            idx = (left + 1, left, left - 1, left - 2)
            w = tuple(-c for c in _ONE_SIDED)    # mirror image: derivative changes sign
        out[..., k] = sum(c * u[..., i] for c, i in zip(w, idx))
    return out


class NCProblem:
    """2D TM PEC cavity on [0,1]^2 advanced by the NC scheme."""

    def __init__(self, n: int, r: float, z: float = 1.0):
        if n < 8:
            raise ValueError("n >= 8")
        self.n, self.r, self.z = n, r, z
        self.h = 1.0 / n
        self.f = {"ez": np.zeros((1, n + 1, n + 1)), "hx": np.zeros((1, n, n + 1)),
                  "hy": np.zeros((1, n + 1, n))}

    def set(self, name, arr):
        a = np.array(arr, dtype=np.float64).reshape(self.f[name].shape)
        if name == "ez":                       # tangential E vanishes on the walls
            a[:, 0, :] = a[:, -1, :] = 0.0
            a[:, :, 0] = a[:, :, -1] = 0.0
        self.f[name] = a

    def get(self, name):
        return self.f[name].copy()

    def step(self, nsteps: int = 1):
        n, h, z = self.n, self.h, self.z
        ht = self.r * h
        for _ in range(nsteps):
            hx, hy, ez = self.f["hx"], self.f["hy"], self.f["ez"]
            # Ez at interior nodes (i, j) = 1 .. n-1: Dx Hy along x (Hy at
            # half points i - 1/2 -> inputs 0 .. n-1), Dy Hx along y
            dxhy = staggered_derivative(hy[:, 1:n, :], n - 1) / h          # (1, n-1, n-1)
            dyhx = np.swapaxes(staggered_derivative(np.swapaxes(hx[:, :, 1:n], 1, 2), n - 1), 1, 2) / h
            ez = ez.copy()
            ez[:, 1:n, 1:n] += ht * z * (dxhy - dyhx)
            # Hx at (i, j + 1/2), i = 1 .. n-1 (the walls i = 0, n keep their
            # values): Dy Ez along y (Ez at nodes 0 .. n -> n outputs)
            dyez = np.swapaxes(staggered_derivative(np.swapaxes(ez[:, :, 1:n], 1, 2), n), 1, 2) / h
            hx = hx.copy()
            hx[:, :, 1:n] -= ht / z * dyez
            # Hy at (i + 1/2, j), j = 1 .. n-1: Dx Ez along x
            dxez = staggered_derivative(ez[:, 1:n, :], n) / h
            hy = hy.copy()
            hy[:, 1:n, :] += ht / z * dxez
            self.f = {"ez": ez, "hx": hx, "hy": hy}
