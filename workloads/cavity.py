"""Closed-form PEC cavity modes sampled on the staggered (Yee) grids.

The 2D TM mode is the paper's analytical solution (Section 5.1, eq:data);
for an impedance Z other than 1 the H amplitude carries a 1/Z so that the
rescaled system (eq:maxwellv) holds with walls at x, y = 0, 1.  The 3D mode
is the cube-cavity analogue: E = e cos(w t) with e orthogonal to k, H from
Faraday's law.

Arrays are (nz, ny, nx), x fastest, walls included; a node axis has N+1
points x_i = i h, a half-point axis N points x_{i+1/2} (eq:meshes).
"""
from __future__ import annotations

import numpy as np

_AXES = "xyz"


def component_names(dim: int):
    return ["ez", "hx", "hy"] if dim == 2 else ["ex", "ey", "ez", "hx", "hy", "hz"]


def component_half_axes(name: str, dim: int):
    """Half-point flag per axis (x, y, z): E_s is at half points along s,
    H_s at half points along the two other axes."""
    s = _AXES.index(name[1])
    half = [False, False, False]
    for a in range(3):
        half[a] = (a == s) if name[0] in "el" else (a != s)
    if dim == 2:
        half[2] = False
    return tuple(half)


def field_shape(name: str, dim: int, n: int):
    half = component_half_axes(name, dim)
    ext = [n if half[a] else n + 1 for a in range(3)]
    if dim == 2:
        ext[2] = 1
    return (ext[2], ext[1], ext[0])


def grid_coords(name: str, dim: int, n: int):
    """Coordinate arrays (z, y, x) broadcastable to field_shape."""
    h = 1.0 / n
    half = component_half_axes(name, dim)
    shp = field_shape(name, dim, n)
    out = []
    for a, size in zip((2, 1, 0), shp):
        c = (np.arange(size) + (0.5 if half[a] else 0.0)) * h
        if dim == 2 and a == 2:
            c = np.zeros(1)
        out.append(c)
    z, y, x = out
    return z[:, None, None], y[None, :, None], x[None, None, :]


def mode_omega(k):
    return np.pi * float(np.sqrt(np.sum(np.asarray(k, dtype=np.float64) ** 2)))


def polarisation_3d(k):
    """Unit E polarisation orthogonal to k: k x (1,1,1), or k x (1,0,0) when k
    is parallel to (1,1,1)."""
    k = np.asarray(k, dtype=np.float64)
    e = np.cross(k, np.ones(3))
    if np.linalg.norm(e) < 1e-12:
        e = np.cross(k, np.array([1.0, 0.0, 0.0]))
    return e / np.linalg.norm(e)


def mode_fields(dim: int, n: int, k, tau_e: float, tau_h: float, amp: float = 1.0,
                z: float = 1.0, with_laplacian: bool = True):
    """Exact mode: E at time tau_e, H at time tau_h; optionally the carried
    Laplacian l = h^2 Delta E at tau_e (zero on the walls)."""
    h = 1.0 / n
    k = tuple(int(v) for v in k)
    w = mode_omega(k)
    out = {}
    if dim == 2:
        kx, ky = k
        zc, yc, xc = grid_coords("ez", 2, n)
        out["ez"] = amp * np.cos(w * tau_e) * np.sin(np.pi * kx * xc) * np.sin(np.pi * ky * yc) + 0 * zc
        zc, yc, xc = grid_coords("hx", 2, n)
        out["hx"] = (-amp * np.pi * ky / (z * w) * np.sin(w * tau_h)
                     * np.sin(np.pi * kx * xc) * np.cos(np.pi * ky * yc) + 0 * zc)
        zc, yc, xc = grid_coords("hy", 2, n)
        out["hy"] = (amp * np.pi * kx / (z * w) * np.sin(w * tau_h)
                     * np.cos(np.pi * kx * xc) * np.sin(np.pi * ky * yc) + 0 * zc)
        if with_laplacian:
            out["lz"] = -(h * np.pi) ** 2 * (kx * kx + ky * ky) * out["ez"]
        return {a: np.ascontiguousarray(v) for a, v in out.items()}
    kv = np.asarray(k, dtype=np.float64)
    e = polarisation_3d(kv)
    c = np.cross(kv, e)
    for s in range(3):
        name = "e" + _AXES[s]
        zc, yc, xc = grid_coords(name, 3, n)
        pat = [np.sin, np.sin, np.sin]
        pat[s] = np.cos
        coords = (xc, yc, zc)
        val = amp * e[s] * np.cos(w * tau_e)
        arr = val * pat[0](np.pi * kv[0] * coords[0]) * pat[1](np.pi * kv[1] * coords[1]) \
            * pat[2](np.pi * kv[2] * coords[2])
        out[name] = np.ascontiguousarray(np.broadcast_to(arr, field_shape(name, 3, n)))
        if with_laplacian:
            out["l" + _AXES[s]] = -(h * np.pi) ** 2 * float(kv @ kv) * out[name]
    for s in range(3):
        name = "h" + _AXES[s]
        zc, yc, xc = grid_coords(name, 3, n)
        pat = [np.cos, np.cos, np.cos]
        pat[s] = np.sin
        coords = (xc, yc, zc)
        val = -amp * np.pi / (z * w) * c[s] * np.sin(w * tau_h)
        arr = val * pat[0](np.pi * kv[0] * coords[0]) * pat[1](np.pi * kv[1] * coords[1]) \
            * pat[2](np.pi * kv[2] * coords[2])
        out[name] = np.ascontiguousarray(np.broadcast_to(arr, field_shape(name, 3, n)))
    return {a: np.ascontiguousarray(v) for a, v in out.items()}
