"""Pins of the oracle's direct transform solve of M (Appendix A.2,
Def. def:operatorsP; oracle/transform_oracle.py).

* It equals a dense solve of M assembled here from the stencil weights
  (the 9-point / 19-point L9 of eq:ell) with the boundary rule of each axis
  (node axis: zero beyond the unknowns; half-point axis: even ghost), for
  every 2D and 3D component at small N.
* It equals the C oracle's CG solve of M (itself pinned by a dense Cholesky
  solve) at larger N, 1e-13.
* The eigenvalue formula: the C oracle's M applied to a product sine /
  cosine mode returns lambda times the mode; every lambda lies in the
  interval [alpha, alpha + (16/3) beta] of Appendix A.1.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import transform_oracle as T
from workloads import component_names, field_shape

W9_2D = {0: -20 / 6, 1: 4 / 6, 2: 1 / 6}          # by the number of non-zero offsets
W19_3D = {0: -24 / 6, 1: 2 / 6, 2: 1 / 6, 3: 0.0}


def dense_m(name, dim, n, r):
    """M on the unknowns as a dense matrix, built point by point."""
    alpha, beta = 1 + 2 / r ** 2, r ** 2 / 24
    kinds = T.axis_kinds(name, dim)
    ranges = []
    for a in range(dim):
        ranges.append(range(1, n) if kinds[a] == "dirichlet" else range(0, n))
    pts = list(itertools.product(*ranges))            # (x, y[, z])
    index = {p: i for i, p in enumerate(pts)}
    w = W9_2D if dim == 2 else W19_3D
    M = np.zeros((len(pts), len(pts)))
    for p in pts:
        for off in itertools.product((-1, 0, 1), repeat=dim):
            q = list(p)
            dropped = False
            for a in range(dim):
                q[a] += off[a]
                lo, hi = ranges[a][0], ranges[a][-1]
                if q[a] < lo or q[a] > hi:
                    if kinds[a] == "dirichlet":
                        dropped = True
                    q[a] = min(max(q[a], lo), hi)
            if dropped:
                continue
            nz = sum(1 for o in off if o)
            lap = w[nz]
            M[index[p], index[tuple(q)]] += (alpha if nz == 0 else 0.0) - beta * lap
    return M, pts


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 11), (3, 8)])
def test_equals_dense_stencil_solve(dim, n):
    rng = np.random.default_rng(dim * 100 + n)
    r = 0.5 if dim == 2 else 0.4
    for name in component_names(dim):
        M, pts = dense_m(name, dim, n, r)
        b = np.zeros(field_shape(name, dim, n))
        vals = rng.normal(size=len(pts))
        for v, p in zip(vals, pts):
            b[(p[2] if dim == 3 else 0, p[1], p[0])] = v
        x = T.solve_m(name, dim, n, r, b)
        ref = np.linalg.solve(M, vals)
        got = np.array([x[(p[2] if dim == 3 else 0, p[1], p[0])] for p in pts])
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)) * 10, name
        # nothing off the unknowns
        mask = np.ones(b.shape, bool)
        mask[T.unknown_slices(name, dim)] = False
        assert not np.any(x[mask])


@pytest.mark.parametrize("dim,n,r", [(2, 40, 0.5), (2, 67, 0.3), (3, 16, 0.4), (3, 21, 0.45)])
def test_equals_oracle_cg_solve(dim, n, r):
    rng = np.random.default_rng(n)
    o = oracle.OracleProblem(dim, n, r, 1.0)
    for name in component_names(dim):
        b = rng.normal(size=field_shape(name, dim, n))
        mask = np.zeros(b.shape, bool)
        mask[T.unknown_slices(name, dim)] = True
        b = np.where(mask, b, 0.0)
        x = T.solve_m(name, dim, n, r, b)
        ref = o.solve_m(name, b)
        assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref), name
        # and M x gives b back through the oracle's own M
        assert np.linalg.norm(o.apply_m(name, x) - b) <= 1e-13 * np.linalg.norm(b), name
    o.close()


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 12)])
def test_eigenvalues_on_modes(dim, n):
    r = 0.5 if dim == 2 else 0.4
    alpha, beta = 1 + 2 / r ** 2, r ** 2 / 24
    o = oracle.OracleProblem(dim, n, r, 1.0)
    rng = np.random.default_rng(7)
    for name in component_names(dim):
        kinds = T.axis_kinds(name, dim)
        lam = T.m_eigenvalues(name, dim, n, r)
        assert lam.min() >= alpha - 1e-12 and lam.max() <= alpha + 16 / 3 * beta + 1e-12
        for _ in range(3):
            mode = np.ones(field_shape(name, dim, n))
            sl = T.unknown_slices(name, dim)
            idx = []
            for a in range(3):
                kd = kinds[a]
                if kd is None:
                    idx.append(0)
                    continue
                m = n - 1 if kd == "dirichlet" else n
                k = int(rng.integers(0, m))
                idx.append(k)
                j = np.arange(field_shape(name, dim, n)[2 - a])
                f = np.sin(np.pi * (k + 1) * j / n) if kd == "dirichlet" else np.cos(np.pi * k * (j + 0.5) / n)
                shp = [1, 1, 1]
                shp[2 - a] = f.size
                mode = mode * f.reshape(shp)
            masked = np.zeros_like(mode)
            masked[sl] = mode[sl]
            got = o.apply_m(name, masked)
            want = lam[idx[2], idx[1], idx[0]] * masked
            assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), (name, idx)
    o.close()
