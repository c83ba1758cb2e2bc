"""Parity of the gfx950 3D stepper (Ex..Hz, through the C ABI) with the CPU
oracle.  Tolerance as in 2D: 1e-12 relative L2 over E and H; the carried
Laplacian at 1e-9 (recovered from G_E = alpha E + l/12 on the device)."""
import numpy as np
import pytest

from gpu_util import rel_l2, rel_l2_all, run_pair

pytestmark = pytest.mark.gpu

EH = ["ex", "ey", "ez", "hx", "hy", "hz"]


def _check(gf, of, tol=1e-12, lap_tol=1e-9):
    assert rel_l2_all(gf, of, EH) <= tol, {a: rel_l2(gf[a], of[a]) for a in EH}
    scale = max(np.max(np.abs(of[a])) for a in EH)
    for a in EH:
        assert np.max(np.abs(gf[a] - of[a])) <= tol * scale * 10, a
    for a in ("lx", "ly", "lz"):
        if a in gf:
            assert rel_l2(gf[a], of[a]) <= lap_tol, a


@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("n", [8, 13])
def test_mode_parity_3d(closure, lap, n):
    gf, of = run_pair(3, n, 0.4, 6, closure=closure, lap=lap, k=(2, 3, 4))
    _check(gf, of)


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_random_data_parity_3d(lap):
    gf, of = run_pair(3, 11, 0.45, 4, closure="paper", lap=lap, seed=99)
    _check(gf, of)


def test_config3_mode_3d_tiles():
    # mode (2,3,4) with e = (-1,2,-1)/sqrt(6), CFL 0.4; 34 > one 32-output tile
    gf, of = run_pair(3, 34, 0.4, 3, k=(2, 3, 4))
    _check(gf, of)
