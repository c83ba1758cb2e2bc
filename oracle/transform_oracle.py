"""Plain FP64 CPU reference of the direct transform solve of M.

TEST INFRASTRUCTURE ONLY: the product package never imports this module.

M = alpha I - beta L9 (eq:ell, Def. def:operatorsP), alpha = 1 + 2/r^2,
beta = r^2/24, acts on one field component's unknowns.  Written with the
one-dimensional second difference D_d of each active axis (unit spacing,
the component's boundary rule on that axis),
    L9 = sum_d D_d + (1/6) sum_{d<e} D_d D_e
(the 5/7-point Laplacian plus one sixth of the mixed fourth differences:
the 9-point stencil (1/6)[1 4 1; 4 -20 4; 1 4 1] in 2D, centre -24/6,
faces 2/6, edges 1/6 in 3D).  The D_d act on different axes, so they
commute, and each one is diagonal in a fixed basis (Appendix A.2):
  * node axis (Dirichlet: unknowns 1..N-1, zero on the walls): the sine
    modes sin(pi k j / N), k = 1..N-1 (DST-I);
  * half-point axis (Neumann, even ghost at the walls: unknowns 0..N-1):
    the cosine modes cos(pi k (j + 1/2) / N), k = 0..N-1 (DCT-II);
both with eigenvalue -sigma_k, sigma_k = 4 sin^2(pi k / (2N)).  Hence M is
diagonal in the product basis with
    lambda = alpha + beta (sum_d sigma_d - (1/6) sum_{d<e} sigma_d sigma_e),
and M^{-1} b = T^T (T b / lambda) with T the orthonormal DST-I / DCT-II on
each active axis.  Neither the closure rows of A nor the carried Laplacian
enter M, so the solve is exact for both closures.  The FFT-based transforms
of scipy serve as the library steps.

Arrays are the stored component arrays (nz, ny, nx), x fastest, walls
included; entries off the unknowns are ignored on input and zero on output.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sf

_AX = "xyz"


def axis_kinds(name: str, dim: int):
    """Per axis (x, y, z): None (inactive), "dirichlet" or "neumann".  E_s
    and l_s sit at half points along s, H_s at half points along the two
    other axes."""
    s = _AX.index(name[1])
    out = []
    for a in range(3):
        if a >= dim:
            out.append(None)
            continue
        half = (a == s) if name[0] in "el" else (a != s)
        out.append("neumann" if half else "dirichlet")
    return out


def _sigma(kind: str, n: int) -> np.ndarray:
    k = np.arange(1, n) if kind == "dirichlet" else np.arange(n)
    return 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2


def unknown_slices(name: str, dim: int):
    """Slices (z, y, x) of the unknowns inside the stored array."""
    kinds = axis_kinds(name, dim)
    sl = []
    for a in (2, 1, 0):
        kd = kinds[a]
        sl.append(slice(None) if kd is None else (slice(1, -1) if kd == "dirichlet" else slice(None)))
    return tuple(sl)


def m_eigenvalues(name: str, dim: int, n: int, r: float) -> np.ndarray:
    """lambda on the unknown grid, shaped like the unknowns (z, y, x)."""
    alpha, beta = 1.0 + 2.0 / r ** 2, r ** 2 / 24.0
    kinds = axis_kinds(name, dim)
    sig = []
    for a in range(3):
        if kinds[a] is None:
            sig.append(np.zeros(1))
        else:
            sig.append(_sigma(kinds[a], n))
    sx = sig[0][None, None, :]
    sy = sig[1][None, :, None]
    sz = sig[2][:, None, None]
    total = sx + sy + sz
    mixed = sx * sy + sx * sz + sy * sz
    return alpha + beta * (total - mixed / 6.0)


def _forward(u: np.ndarray, kinds) -> np.ndarray:
    for a, kd in enumerate(kinds):
        if kd is None:
            continue
        ax = 2 - a
        u = sf.dst(u, type=1, norm="ortho", axis=ax) if kd == "dirichlet" else sf.dct(u, type=2, norm="ortho", axis=ax)
    return u


def _inverse(u: np.ndarray, kinds) -> np.ndarray:
    for a, kd in enumerate(kinds):
        if kd is None:
            continue
        ax = 2 - a
        u = sf.idst(u, type=1, norm="ortho", axis=ax) if kd == "dirichlet" else sf.idct(u, type=2, norm="ortho", axis=ax)
    return u


def solve_m(name: str, dim: int, n: int, r: float, b: np.ndarray) -> np.ndarray:
    """x = M^{-1} b on the unknowns of component `name` (stored layout)."""
    kinds = axis_kinds(name, dim)
    sl = unknown_slices(name, dim)
    bu = np.asarray(b, dtype=np.float64)[sl]
    xu = _inverse(_forward(bu, kinds) / m_eigenvalues(name, dim, n, r), kinds)
    x = np.zeros(np.shape(b))
    x[sl] = xu
    return x
