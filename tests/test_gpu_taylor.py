"""Taylor start of H on the device (Section 5.1, eq:talorh, J = 0) against
the oracle's: H(h_tau/2) from E and H at tau = 0, then steps of the scheme
from it, 2D and 3D, both closures, random data with non-zero normal-H walls
(kept) and sizes spanning several line tiles with ragged tails.  The call is
refused once a step has been taken and for the NC scheme.
"""
import numpy as np
import pytest

import oracle
from gpu_util import CLOSURES, LAPS, check_fields, random_fields

pytestmark = pytest.mark.gpu


def _pair(dim, n, r, z, closure, lap):
    from paper_2306_17263_amd import Problem
    g = Problem(dim, n, r, z=z, closure=closure, lap_mode=lap)
    o = oracle.OracleProblem(dim, n, r, z, closure=CLOSURES[closure], lap_mode=LAPS[lap])
    return g, o


@pytest.mark.parametrize("dim,n,r,z", [(2, 8, 0.5, 1.0), (2, 77, 0.5, 1.3), (2, 300, 0.4, 0.8),
                                       (3, 8, 0.4, 1.0), (3, 21, 0.4, 1.7), (3, 66, 0.3, 1.0)])
@pytest.mark.parametrize("closure", ["paper", "reflect"])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_taylor_start_matches_oracle(dim, n, r, z, closure, lap):
    g, o = _pair(dim, n, r, z, closure, lap)
    init = random_fields(dim, n, seed=1000 * dim + n, h_walls=True)
    for name in g.fields():
        g.set(name, init[name])
        o.set(name, init[name])
    g.init_h_taylor()
    o.init_h_taylor()
    names = g.fields()
    gf = {a: g.get(a) for a in names}
    of = {a: o.get(a) for a in names}
    check_fields(gf, of)
    # normal-H wall values and E are unchanged
    for a in names:
        if a[0] in "el":
            assert np.array_equal(gf[a], init[a]) or a[0] == "l", a
    for a in names:
        if a[0] == "h":
            ax = "xyz".index(a[1])
            for idx in (0, -1):
                sl = [slice(None)] * 3
                sl[2 - ax] = idx
                assert np.array_equal(gf[a][tuple(sl)], init[a][tuple(sl)]), a
    g.step(3)
    o.step(3)
    check_fields({a: g.get(a) for a in names}, {a: o.get(a) for a in names})
    g.close()


def test_taylor_start_refused_after_step_and_for_nc():
    from paper_2306_17263_amd import C4mError, Problem
    g = Problem(2, 16, 0.5)
    g.step(1)
    with pytest.raises(C4mError):
        g.init_h_taylor()
    g.close()
    g = Problem(2, 16, 0.5, scheme="nc")
    with pytest.raises(C4mError):
        g.init_h_taylor()
    g.close()
