"""Pins of the oracle's compact elliptic operator M = alpha I - beta L9
(eq:ell scaled by h_tau^2/24, Definition def:operatorsP) and its CG solve.

* Dense assembly from the one-dimensional second-difference matrices of
  Appendix A.1 (Dirichlet along node axes, even ghost along half axes, as in
  Table tab:bc and Corollary cor:ghost_cor) and a Cholesky solve.
* Closed-form eigenvalue on sampled sine/cosine modes.
* Spectrum inside [alpha, alpha + (16/3) beta] (the operator estimates of
  Appendix A.2 with the exact range of the symbol S).
"""
import numpy as np
import pytest

import oracle
from workloads import component_half_axes, field_shape

DIM_FIELDS = {2: ["ez", "hx", "hy"], 3: ["ex", "ey", "ez", "hx", "hy", "hz"]}


def _d2_1d(n, half):
    """Second difference on the unknowns of one axis."""
    m = n if half else n - 1
    a = -2.0 * np.eye(m) + np.eye(m, k=1) + np.eye(m, k=-1)
    if half:                       # even ghost folds onto the boundary unknown
        a[0, 0] = a[-1, -1] = -1.0
    return a


def _dense_m(name, dim, n, r):
    alpha, beta = 1 + 2 / r ** 2, r ** 2 / 24
    half = component_half_axes(name, dim)
    mats = [_d2_1d(n, half[a]) for a in range(dim)]          # x, y, (z)
    eyes = [np.eye(m.shape[0]) for m in mats]

    def kron_axes(ops):                                       # ops indexed by axis, x fastest
        out = np.array([[1.0]])
        for a in reversed(range(dim)):
            out = np.kron(out, ops[a])
        return out

    lap = sum(kron_axes([mats[a] if a == b else eyes[a] for a in range(dim)]) for b in range(dim))
    mixed = 0
    for d in range(dim):
        for e in range(d + 1, dim):
            mixed = mixed + kron_axes([mats[a] if a in (d, e) else eyes[a] for a in range(dim)])
    l9 = lap + mixed / 6.0
    return alpha * np.eye(l9.shape[0]) - beta * l9


def _unknown_slices(name, dim, n):
    half = component_half_axes(name, dim)
    sl = []
    for a in (2, 1, 0):
        if a >= dim:
            sl.append(slice(0, 1))
        else:
            sl.append(slice(0, n) if half[a] else slice(1, n))
    return tuple(sl)


@pytest.mark.parametrize("dim,n,r", [(2, 8, 0.5), (2, 11, 0.589), (3, 8, 0.4)])
def test_solve_matches_dense_cholesky(dim, n, r):
    p = oracle.OracleProblem(dim, n, r)
    rng = np.random.default_rng(dim * 100 + n)
    for name in DIM_FIELDS[dim]:
        mdense = _dense_m(name, dim, n, r)
        chol = np.linalg.cholesky(mdense)                      # SPD, else this raises
        sl = _unknown_slices(name, dim, n)
        b = np.zeros(field_shape(name, dim, n))
        b[sl] = rng.normal(size=b[sl].shape)
        y = np.linalg.solve(chol.T, np.linalg.solve(chol, b[sl].ravel()))
        x = p.solve_m(name, b)
        assert np.max(np.abs(x[sl].ravel() - y)) <= 1e-13 * np.max(np.abs(y)), name
        # and the stencil itself equals the dense matrix
        mx = p.apply_m(name, x)
        assert np.max(np.abs(mx[sl].ravel() - mdense @ x[sl].ravel())) <= 1e-13 * np.max(np.abs(b))
        # walls stay zero
        mask = np.ones(b.shape, bool)
        mask[sl] = False
        assert np.all(x[mask] == 0.0)


@pytest.mark.parametrize("dim,r", [(2, 0.5), (3, 0.4)])
def test_mode_eigenvalue(dim, r):
    n = 12
    h = 1.0 / n
    alpha, beta = 1 + 2 / r ** 2, r ** 2 / 24
    p = oracle.OracleProblem(dim, n, r)
    rng = np.random.default_rng(5)
    for name in DIM_FIELDS[dim]:
        half = component_half_axes(name, dim)
        for _ in range(4):
            ks = [int(rng.integers(0 if half[a] else 1, n)) for a in range(dim)]
            shp = field_shape(name, dim, n)
            grids = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")   # z, y, x
            mode = np.ones(shp)
            for a in range(dim):
                idx = grids[2 - a]
                if half[a]:
                    mode *= np.cos(np.pi * ks[a] * (idx + 0.5) * h)
                else:
                    mode *= np.sin(np.pi * ks[a] * idx * h)
            sig = [4 * np.sin(np.pi * k * h / 2) ** 2 for k in ks]
            mixed = sum(sig[a] * sig[b] for a in range(dim) for b in range(a + 1, dim))
            lam = alpha + beta * (sum(sig) - mixed / 6)
            got = p.apply_m(name, mode)
            sl = _unknown_slices(name, dim, n)
            assert np.max(np.abs(got[sl] - lam * mode[sl])) < 1e-12 * lam, (name, ks)


@pytest.mark.parametrize("dim,n,r", [(2, 9, 0.5), (3, 8, 0.4)])
def test_spectrum_bounds(dim, n, r):
    alpha, beta = 1 + 2 / r ** 2, r ** 2 / 24
    for name in DIM_FIELDS[dim]:
        ev = np.linalg.eigvalsh(_dense_m(name, dim, n, r))
        assert ev.min() >= alpha - 1e-12
        assert ev.max() <= alpha + 16 / 3 * beta + 1e-12


def test_cg_iterations_are_few():
    # the Conclusions report about three CG iterations independent of N
    for n in (32, 64, 128):
        p = oracle.OracleProblem(2, n, 0.5, rtol=1e-12)
        rng = np.random.default_rng(n)
        b = rng.normal(size=field_shape("ez", 2, n))
        x = p.solve_m("ez", b)
        assert np.all(np.isfinite(x))
    from workloads import mode_fields
    for n in (32, 64, 128):
        p = oracle.OracleProblem(2, n, 0.5, rtol=1e-12)
        f = mode_fields(2, n, (4, 3), 0.0, 0.25 / n)
        for k, v in f.items():
            p.set(k, v)
        p.step(4)
        last, mx = p.cg_stats()
        assert mx <= 5
