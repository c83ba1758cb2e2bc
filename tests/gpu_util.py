"""Helpers shared by the GPU parity tests: run the same seeded problem on the
device (through the C ABI) and on the CPU oracle, and compare."""
from __future__ import annotations

import numpy as np

import oracle
from workloads import mode_fields

CLOSURES = {"paper": oracle.CLOSURE_PAPER, "reflect": oracle.CLOSURE_REFLECT}
LAPS = {"tracked": oracle.LAP_TRACKED, "discrete": oracle.LAP_DISCRETE}


def initial_fields(dim, n, cfl, k=None, seed=None, amp=1.0, z=1.0):
    """Exact cavity mode (k given) or seeded random data with PEC walls."""
    h = 1.0 / n
    if k is not None:
        return mode_fields(dim, n, k, 0.0, cfl * h / 2, amp=amp, z=z)
    from workloads import component_names, field_shape
    rng = np.random.default_rng(seed)
    out = {}
    for name in component_names(dim):
        a = rng.normal(size=field_shape(name, dim, n))
        if name[0] == "h":                       # normal H on its walls: zero
            ax = "xyz".index(name[1])
            sl = [slice(None)] * 3
            sl[2 - ax] = 0
            a[tuple(sl)] = 0.0
            sl[2 - ax] = -1
            a[tuple(sl)] = 0.0
        out[name] = a
    for name in list(out):
        if name[0] == "e":
            out["l" + name[1]] = 0.1 * rng.normal(size=out[name].shape)
    return out


def run_pair(dim, n, cfl, steps, closure="paper", lap="tracked", k=(1, 1), seed=None, z=1.0, **kw):
    """Returns (gpu_fields, oracle_fields) after `steps` steps."""
    from paper_2306_17263_amd import Problem
    init = initial_fields(dim, n, cfl, k=k if seed is None else None, seed=seed, z=z)
    g = Problem(dim, n, cfl, z=z, closure=closure, lap_mode=lap, **kw)
    o = oracle.OracleProblem(dim, n, cfl, z, closure=CLOSURES[closure], lap_mode=LAPS[lap])
    for name in g.fields():
        g.set(name, init[name])
        o.set(name, init[name])
    g.step(steps)
    o.step(steps)
    gf = {name: g.get(name) for name in g.fields()}
    of = {name: o.get(name) for name in g.fields()}
    g.close()
    return gf, of


def rel_l2(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def rel_l2_all(gf, of, names):
    num = sum(np.sum((gf[a] - of[a]) ** 2) for a in names)
    den = sum(np.sum(of[a] ** 2) for a in names)
    return float(np.sqrt(num / den))
