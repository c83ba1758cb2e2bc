"""Writes convergence_mode43_t1.txt: the CPU oracle's relative L2 error
against the exact cavity mode (4, 3) after T = 1 at CFL 0.5 (E at T, H at
T + h_tau/2, over Ez, Hx, Hy), for N = 64, 128, 256, both closures, carried
Laplacian.  Calls only the oracle; the exact mode is eq:data (Section 5.1).

    python tests/golden/make_convergence.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import mode_fields  # noqa: E402

NAMES = ["ez", "hx", "hy"]


def oracle_error(n, closure, k=(4, 3), cfl=0.5):
    ht = cfl / n
    steps = int(round(1.0 / ht))
    init = mode_fields(2, n, k, 0.0, ht / 2)
    o = oracle.OracleProblem(2, n, cfl, 1.0, closure=closure, lap_mode=oracle.LAP_TRACKED)
    for name in NAMES + ["lz"]:
        o.set(name, init[name])
    o.step(steps)
    ex = mode_fields(2, n, k, steps * ht, (steps + 0.5) * ht)
    num = sum(float(np.sum((o.get(a) - ex[a]) ** 2)) for a in NAMES)
    den = sum(float(np.sum(ex[a] ** 2)) for a in NAMES)
    return float(np.sqrt(num / den))


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "convergence_mode43_t1.txt")
    lines = ["# closure n rel_l2 (oracle, mode (4,3), CFL 0.5, T = 1, carried Laplacian)"]
    for cname, closure in (("paper", oracle.CLOSURE_PAPER), ("reflect", oracle.CLOSURE_REFLECT)):
        for n in (64, 128, 256):
            lines.append(f"{cname} {n} {oracle_error(n, closure):.12e}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
