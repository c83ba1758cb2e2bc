"""Seeded problem mixes for the batched and serving forms.

Batch mix: independent 2D TM cavities, N uniform in [n_lo, n_hi], modes
(k, l) uniform in 1..8, amplitude uniform in (0.5, 2), CFL 0.5.
Serving mix: Poisson arrivals at a fixed rate, half 2D (N in 64..1024) and
half 3D (N in 32..128), 100..2000 steps each, random modes.
"""
from __future__ import annotations

import numpy as np


def batch_mix(count: int = 512, seed: int = 2306, n_lo: int = 64, n_hi: int = 768,
              kmax: int = 8, steps: int = 200, r: float = 0.5):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        k = (int(rng.integers(1, kmax + 1)), int(rng.integers(1, kmax + 1)))
        amp = float(rng.uniform(0.5, 2.0))
        out.append({"dim": 2, "n": n, "k": k, "amp": amp, "steps": steps, "r": r})
    return out


def serving_arrivals(count: int = 2000, seed: int = 17263, rate: float = 200.0,
                     frac_3d: float = 0.5, n2: tuple = (64, 1024), n3: tuple = (32, 128),
                     steps: tuple = (100, 2000), kmax: int = 8):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        dim = 3 if rng.uniform() < frac_3d else 2
        lo, hi = n3 if dim == 3 else n2
        n = int(rng.integers(lo, hi + 1))
        k = tuple(int(rng.integers(1, kmax + 1)) for _ in range(dim))
        out.append({"id": i, "t_arrive": t, "dim": dim, "n": n, "k": k,
                    "amp": float(rng.uniform(0.5, 2.0)),
                    "steps": int(rng.integers(steps[0], steps[1] + 1)),
                    "r": 0.4 if dim == 3 else 0.5})
    return out
