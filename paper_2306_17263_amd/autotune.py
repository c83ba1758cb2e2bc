"""Autotuner for the kernel launch shape.

Tunables (fields of c4m_config):
  tile_x  column-kernel shape.  Single 2D problems: 0 = wave strips (one
          wavefront per 64 columns streaming down a row segment, 8 steps
          per unrolled block), 4 = wave strips with 16 steps per block,
          1 = 64 x 4 column tiles, 2 = 128 x 2, 3 = 128 x 4.  Batched form:
          0 = 128 columns x 4 lanes per column, 1 = 64 x 4, 2 = 128 x 2
          (shapes 1 and 2 exist for 4..6 sweeps);
  tile_y  batched form only: persistent-grid multiplier (workgroups per
          launch = multiplier x what fits on the device at once).
The halo depth of the column tiles equals the number of Chebyshev sweeps,
which the accuracy target fixes (the smallest count reaching 4e-16 on the
spectral bounds of M); the tuner keeps it and picks the shape.

Candidates are timed on the caller's workload with HIP events on a private
stream; the winner is cached in a JSON file keyed by device, dimension,
size bucket and settings (C4M_TUNE_CACHE, default ~/.cache/c4m_autotune.json).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "c4m_autotune.json")
SHAPES = (0, 1, 2)            # batched form
SINGLE_SHAPES = (0, 4, 3)     # single 2D problems: strips, strips x16, 128 x 4 tiles
GRID_MULT = (1, 2)


def cache_path() -> str:
    return os.environ.get("C4M_TUNE_CACHE", DEFAULT_CACHE)


def size_bucket(n: int) -> int:
    """Power-of-two bucket of the grid size."""
    b = 16
    while b < n:
        b *= 2
    return b


def make_key(device: str, kind: str, dim: int, n: int, settings: dict) -> str:
    s = ",".join(f"{k}={settings[k]}" for k in sorted(settings))
    return f"{device}|{kind}|d{dim}|n{size_bucket(n)}|{s}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(key: str, value: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = value
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick_best(timings: dict) -> tuple:
    """timings: {candidate: seconds}; the fastest candidate (ties: first)."""
    return min(timings.items(), key=lambda kv: kv[1])[0]


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0).replace("|", "/")


def _time_steps(step, sync, steps: int, reps: int = 2) -> float:
    best = float("inf")
    for _ in range(reps):
        sync()
        t = time.perf_counter()
        step(steps)
        sync()
        best = min(best, time.perf_counter() - t)
    return best


def tune_single(n: int, dim: int = 2, cfl: float = 0.5, steps: int = 8, use_cache: bool = True,
                **settings) -> dict:
    """Best {tile_x} for one problem of size n with the given settings."""
    import torch
    from .problem import Problem
    key = make_key(_device_name(), "single", dim, n, dict(settings, cfl=cfl))
    if use_cache:
        hit = load_cache().get(key)
        if hit:
            return hit
    st = torch.cuda.Stream()
    timings = {}
    # the 3D path and the FP32-refined form have one column-tile shape
    shapes = SINGLE_SHAPES if dim == 2 and settings.get("precision", "fp64") == "fp64" else (0,)
    for shape in shapes:
        p = Problem(dim, n, cfl, stream=st, tile_x=shape, **settings)
        p.step(1)
        timings[shape] = _time_steps(p.step, st.synchronize, steps)
        p.close()
    best = pick_best(timings)
    out = {"tile_x": int(best), "seconds_per_step": timings[best] / steps,
           "timings": {str(k): v / steps for k, v in timings.items()}}
    if use_cache:
        store_cache(key, out)
    return out


def tune_batch(specs, steps: int = 4, use_cache: bool = True, **settings) -> dict:
    """Best {tile_x, tile_y} for a batch of 2D problems (list of {"n": ...})."""
    import torch
    from .batch import Batch
    nmax = max(s["n"] for s in specs)
    key = make_key(_device_name(), f"batch{len(specs)}", 2, nmax, settings)
    if use_cache:
        hit = load_cache().get(key)
        if hit:
            return hit
    st = torch.cuda.Stream()
    timings = {}
    shapes = SHAPES if settings.get("precision", "fp64") == "fp64" else (0,)
    for shape in shapes:
        for mult in GRID_MULT:
            b = Batch(specs, stream=st, tile_x=shape, tile_y=mult, **settings)
            b.step(1)
            timings[(shape, mult)] = _time_steps(b.step, st.synchronize, steps)
            b.close()
    best = pick_best(timings)
    out = {"tile_x": int(best[0]), "tile_y": int(best[1]), "seconds_per_step": timings[best] / steps,
           "timings": {f"{k[0]},{k[1]}": v / steps for k, v in timings.items()}}
    if use_cache:
        store_cache(key, out)
    return out
