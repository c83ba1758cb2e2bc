"""Parity of the gfx950 3D stepper (Ex..Hz, through the C ABI) with the CPU
oracle.  Tolerance as in 2D: 1e-12 relative L2 over E and H, every element
within 1e-11 of the field scale; the carried Laplacian at 1e-9 (recovered
from G_E = alpha E + l/12 on the device).

Lines of at most 48 outputs use exact rows of the truncated Pade inverse
throughout; longer lines (n >= 50) use the Toeplitz interior taps between
the two end bands of 24 rows (Appendix A.1), so the sizes 56, 64 and 72
put the interior branch of the line-term kernel on the oracle for both line
kinds (node -> half with n outputs, half -> node with n - 1)."""
import pytest

from gpu_util import check_fields, run_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("n", [8, 13])
def test_mode_parity_3d(closure, lap, n):
    gf, of = run_pair(3, n, 0.4, 6, closure=closure, lap=lap, k=(2, 3, 4))
    check_fields(gf, of)


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_random_data_parity_3d(lap):
    gf, of = run_pair(3, 11, 0.45, 4, closure="paper", lap=lap, seed=99)
    check_fields(gf, of)


def test_config3_mode_3d_tiles():
    # mode (2,3,4) with e = (-1,2,-1)/sqrt(6), CFL 0.4; 34 > one 32-output tile
    gf, of = run_pair(3, 34, 0.4, 3, k=(2, 3, 4))
    check_fields(gf, of)


@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("n", [56, 64])
def test_interior_taps_parity_3d(closure, lap, n):
    # lines longer than 48 outputs: interior Toeplitz taps between the bands
    gf, of = run_pair(3, n, 0.4, 3, closure=closure, lap=lap, k=(2, 3, 4))
    check_fields(gf, of)


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_interior_taps_random_3d(lap):
    # rough data excite every tap of the interior rows; n = 72 has several
    # interior segments per line
    gf, of = run_pair(3, 72, 0.4, 2, closure="paper", lap=lap, seed=72)
    check_fields(gf, of)


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
def test_interior_taps_fp32_refined_3d(lap, closure):
    gf, of = run_pair(3, 64, 0.4, 3, closure=closure, lap=lap, k=(2, 3, 4), precision="fp32_refined")
    check_fields(gf, of, tol=1e-10, lap_tol=1e-7)


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
def test_interior_taps_pcg_3d(lap, closure):
    gf, of = run_pair(3, 64, 0.4, 3, closure=closure, lap=lap, k=(2, 3, 4), solver="pcg")
    check_fields(gf, of)


def test_full_size_3d_one_step():
    """N = 256 (the 3D workload's size, CFL 0.4, FP64 Chebyshev, the recorded
    step the bench times): one step of seeded random data against the
    oracle, element by element."""
    gf, of = run_pair(3, 256, 0.4, 1, closure="paper", lap="tracked", seed=256)
    check_fields(gf, of)
