"""The sourced 2D step (c4m_step_source: J = (0, 0, Jz), Section 3.1 and
Table tab:spec, ghost values by Method 2, eq:gst2) against the sourced
oracle: seeded random source data and the driven-cavity data, both Laplacian
modes, several impedances, sizes spanning several tiles with ragged edges,
the other solvers and the refined precision; zero sources equal the plain
step bit for bit; on the driven cavity the device errors equal the
oracle's and fall at fourth order; refusals."""
import numpy as np
import pytest

from gpu_util import LAPS, check_fields
from oracle.source_oracle import SourcedTM
from workloads.driven import DrivenTM

pytestmark = pytest.mark.gpu

NAMES = ("ez", "hx", "hy")


def _random_data(n, rng):
    e = lambda: rng.standard_normal((1, n + 1, n + 1))
    w = lambda: [[rng.standard_normal(n + 1), rng.standard_normal(n + 1)] for _ in range(2)]
    d1 = {"jz": e(), "jz_tt": e(), "jz_lap": e(), "jz_tt_lap": e(), "hx_wall": w(), "hy_wall": w()}
    d2 = {"jz_t": e(), "kx": rng.standard_normal((1, n, n + 1)), "kx_lap": rng.standard_normal((1, n, n + 1)),
          "ky": rng.standard_normal((1, n + 1, n)), "ky_lap": rng.standard_normal((1, n + 1, n)),
          "dhx_wall": w(), "dhy_wall": w()}
    return d1, d2


def _pair(n, r, z, lap, init, data, steps, **kw):
    """GPU and oracle fields after `steps` sourced steps; data(m) gives the
    step's (d1, d2)."""
    from paper_2306_17263_amd import Problem
    g = Problem(2, n, r, z=z, lap_mode=lap, **kw)
    s = SourcedTM(n, r, z, LAPS[lap])
    for k in ("ez", "hx", "hy", "lz"):
        if k == "lz" and lap != "tracked":
            continue
        g.set(k, init[k])
        s.set(k, init[k])
    if lap != "tracked":
        s.set("lz", np.zeros_like(init["ez"]))
    for m in range(steps):
        d1, d2 = data(m)
        dd = dict(d1)
        dd.update(d2)
        g.step_source(dd)
        s.step(d1, d2)
    gf = {k: g.get(k) for k in NAMES}
    of = {k: s.get(k) for k in NAMES}
    if lap == "tracked":
        gf["lz"], of["lz"] = g.get("lz"), s.get("lz")
    g.close()
    s.close()
    return gf, of


def _random_init(n, seed):
    rng = np.random.default_rng(seed)
    f = {"ez": rng.standard_normal((1, n + 1, n + 1)), "hx": rng.standard_normal((1, n, n + 1)),
         "hy": rng.standard_normal((1, n + 1, n)), "lz": rng.standard_normal((1, n + 1, n + 1))}
    for k in ("ez", "lz"):
        f[k][:, 0, :] = f[k][:, -1, :] = 0.0
        f[k][:, :, 0] = f[k][:, :, -1] = 0.0
    f["hx"][:, :, 0] = f["hx"][:, :, -1] = 0.0
    f["hy"][:, 0, :] = f["hy"][:, -1, :] = 0.0
    return f


@pytest.mark.parametrize("n", [24, 40, 97, 130])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_random_sources_match_oracle(n, lap):
    rng = np.random.default_rng(1000 + n)
    data = [_random_data(n, rng) for _ in range(3)]
    gf, of = _pair(n, 0.5, 1.3, lap, _random_init(n, n), lambda m: data[m], 3)
    check_fields(gf, of)


@pytest.mark.parametrize("z", [1.0, 1.7])
@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_driven_cavity_matches_oracle(z, lap):
    n, r = 64, 0.5
    drv = DrivenTM(z=z)
    ht = r / n
    init = drv.fields(n, 0.0, ht / 2)
    gf, of = _pair(n, r, z, lap, init, lambda m: (drv.step1_data(n, (m + 0.5) * ht),
                                                   drv.step2_data(n, (m + 1) * ht)), 8)
    check_fields(gf, of)


@pytest.mark.parametrize("kw,tol", [({"solver": "pcg"}, 1e-12), ({"solver": "transform"}, 1e-12),
                                    ({"precision": "fp32_refined"}, 1e-10), ({"tile_x": 2}, 1e-12)])
def test_other_forms_match_oracle(kw, tol):
    n = 40
    rng = np.random.default_rng(7)
    data = [_random_data(n, rng) for _ in range(2)]
    gf, of = _pair(n, 0.5, 1.0, "tracked", _random_init(n, 3), lambda m: data[m], 2, **kw)
    check_fields(gf, of, tol=tol, lap_tol=max(1e-9, 100 * tol))


def test_zero_sources_equal_plain_step():
    from paper_2306_17263_amd import Problem
    n = 72
    init = _random_init(n, 11)
    a = Problem(2, n, 0.5)
    b = Problem(2, n, 0.5)
    for k in ("ez", "hx", "hy", "lz"):
        a.set(k, init[k])
        b.set(k, init[k])
    for _ in range(3):
        a.step_source({})
    b.step(3)
    for k in ("ez", "hx", "hy", "lz"):
        assert np.array_equal(a.get(k), b.get(k)), k
    a.close()
    b.close()


def test_driven_cavity_fourth_order_on_device():
    from paper_2306_17263_amd import Problem
    r, T = 0.5, 0.25
    drv = DrivenTM(z=1.2)
    errs = []
    for n in (16, 32, 64):
        ht = r / n
        steps = int(round(T / ht))
        g = Problem(2, n, r, z=drv.z)
        init = drv.fields(n, 0.0, ht / 2)
        for k in ("ez", "hx", "hy", "lz"):
            g.set(k, init[k])
        for m in range(steps):
            dd = dict(drv.step1_data(n, (m + 0.5) * ht))
            dd.update(drv.step2_data(n, (m + 1) * ht))
            g.step_source(dd)
        fe = drv.fields(n, steps * ht, (steps + 0.5) * ht)
        errs.append(max(np.max(np.abs(g.get(k) - fe[k])) for k in NAMES))
        g.close()
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 4.0, (errs, rates)


def test_full_size_one_step():
    """N = 2048 (the 2D workload size): one sourced step of seeded data
    against the oracle, element by element."""
    n = 2048
    rng = np.random.default_rng(2048)
    data = [_random_data(n, rng)]
    gf, of = _pair(n, 0.5, 1.0, "tracked", _random_init(n, 5), lambda m: data[m], 1)
    check_fields(gf, of)


def test_refusals():
    import ctypes

    from paper_2306_17263_amd import C4mError, Problem
    from paper_2306_17263_amd import _lib as L
    for kw in ({"closure": "reflect"}, {"scheme": "nc"}):
        p = Problem(2, 16, 0.5, **kw)
        with pytest.raises(C4mError):
            p.step_source({})
        p.close()
    p = Problem(3, 8, 0.4)
    with pytest.raises(C4mError):
        p.step_source({})
    p.close()
    p = Problem(2, 16, 0.5)
    lib = L.load()
    need = lib.c4m_source_work_bytes(p._h)
    assert need > 0
    src = L.C4mSourceTM()
    import torch
    w = torch.empty(need, dtype=torch.uint8, device=p.device)
    assert lib.c4m_step_source(p._h, ctypes.byref(src), ctypes.c_void_p(w.data_ptr()), need - 8) != 0
    assert lib.c4m_step_source(p._h, ctypes.byref(src), ctypes.c_void_p(w.data_ptr() + 8), need - 8) != 0
    assert lib.c4m_step_source(p._h, ctypes.byref(src), ctypes.c_void_p(w.data_ptr()), need) == 0
    torch.cuda.synchronize()
    p.close()


def test_check_finite_flag():
    """With C4M_FLAG_CHECK_FINITE a sourced step scans the fields: an
    infinite source value gives ENONFINITE (sticky), finite data passes."""
    from paper_2306_17263_amd import ENONFINITE, FLAG_CHECK_FINITE, C4mError, Problem
    n = 24
    init = _random_init(n, 4)
    p = Problem(2, n, 0.5, flags=FLAG_CHECK_FINITE)
    for k in ("ez", "hx", "hy", "lz"):
        p.set(k, init[k])
    rng = np.random.default_rng(4)
    d1, d2 = _random_data(n, rng)
    good = dict(d1)
    good.update(d2)
    p.step_source(good)
    assert p.info()["nonfinite"] == 0
    bad = dict(good)
    jz = good["jz"].copy()
    jz[0, n // 2, n // 2] = np.inf
    bad["jz"] = jz
    with pytest.raises(C4mError) as ei:
        p.step_source(bad)
    assert ei.value.status == ENONFINITE
    assert p.info()["nonfinite"] == 1
    p.close()


def test_work_buffer_kept_between_calls():
    """The tables go to a work buffer on its first call; later calls reuse
    them, a new buffer gets them again, and the results do not depend on
    which: three steps with one buffer equal three steps alternating two."""
    import ctypes

    import torch

    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd import _lib as L
    n = 40
    init = _random_init(n, 21)
    rng = np.random.default_rng(21)
    data = [_random_data(n, rng) for _ in range(3)]
    out = []
    for alternate in (False, True):
        p = Problem(2, n, 0.5)
        for k in ("ez", "hx", "hy", "lz"):
            p.set(k, init[k])
        lib = L.load()
        need = lib.c4m_source_work_bytes(p._h)
        bufs = [torch.empty(need, dtype=torch.uint8, device=p.device) for _ in range(2)]
        keep = []
        for m in range(3):
            dd = dict(data[m][0])
            dd.update(data[m][1])
            src = L.C4mSourceTM()
            for name in Problem.SOURCE_ARRAYS:
                t = torch.as_tensor(dd[name]).to(p.device).contiguous()
                keep.append(t)
                setattr(src, name, t.data_ptr())
            for name in Problem.SOURCE_WALLS:
                slot = getattr(src, name)
                for w in (0, 1):
                    for d in (0, 1):
                        t = torch.as_tensor(dd[name][w][d]).to(p.device).contiguous()
                        keep.append(t)
                        slot[w][d] = t.data_ptr()
            wb = bufs[m % 2] if alternate else bufs[0]
            assert lib.c4m_step_source(p._h, ctypes.byref(src), ctypes.c_void_p(wb.data_ptr()), need) == 0
        out.append({k: p.get(k) for k in ("ez", "hx", "hy")})
        p.close()
    for k in ("ez", "hx", "hy"):
        assert np.array_equal(out[0][k], out[1][k]), k
