"""ctypes binding of the C oracle (``c4_oracle.c``).  Test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c4_oracle.c")
_LIB = os.path.join(_HERE, "libc4oracle.so")

CLOSURE_PAPER, CLOSURE_REFLECT = 0, 1
LAP_TRACKED, LAP_DISCRETE = 0, 1
FIELDS = {"ex": 0, "ey": 1, "ez": 2, "hx": 3, "hy": 4, "hz": 5, "lx": 6, "ly": 7, "lz": 8}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP over independent lines)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    lib.oc_create.restype = P
    lib.oc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oc_destroy.argtypes = [P]
    lib.oc_field_shape.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.oc_set_field.argtypes = [P, ctypes.c_int, D]
    lib.oc_get_field.argtypes = [P, ctypes.c_int, D]
    lib.oc_step.argtypes = [P, ctypes.c_long]
    lib.oc_half_step_e.argtypes = [P, ctypes.c_double]
    lib.oc_half_step_h.argtypes = [P, ctypes.c_double]
    lib.oc_cg_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.oc_pade_line.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, D, D]
    lib.oc_apply_m.argtypes = [P, ctypes.c_int, D, D]
    lib.oc_solve_m.argtypes = [P, ctypes.c_int, D, D]
    lib.oc_rhs.argtypes = [P, ctypes.c_int, D]
    lib.oc_init_h_taylor.argtypes = [P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pade_line(f, closure: int, node_to_half: bool) -> np.ndarray:
    """A^{-1} D f along one line (no 1/h), eq:lhs."""
    lib = load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(f.size - 1)
    rc = lib.oc_pade_line(f.size, closure, int(node_to_half), _ptr(f), _ptr(out))
    if rc:
        raise ValueError(f"oc_pade_line failed ({rc})")
    return out


class OracleProblem:
    """One cavity problem held by the C oracle.  Arrays are (nz, ny, nx)."""

    def __init__(self, dim: int, n: int, r: float, z: float = 1.0,
                 closure: int = CLOSURE_PAPER, lap_mode: int = LAP_TRACKED,
                 rtol: float = 1e-15, max_iter: int = 100):
        self._lib = load()
        self.dim, self.n, self.r, self.z = dim, n, r, z
        self.closure, self.lap_mode = closure, lap_mode
        self._p = self._lib.oc_create(dim, n, r, z, closure, lap_mode, rtol, max_iter)
        if not self._p:
            raise ValueError("oc_create rejected the configuration")

    def close(self):
        if self._p:
            self._lib.oc_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fields(self):
        names = ["ez", "hx", "hy", "lz"] if self.dim == 2 else list(FIELDS)
        return names

    def shape(self, name: str):
        s = (ctypes.c_int * 3)()
        if self._lib.oc_field_shape(self._p, FIELDS[name], s):
            raise KeyError(name)
        return (s[2], s[1], s[0])

    def set(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.shape(name))
        if self._lib.oc_set_field(self._p, FIELDS[name], _ptr(a)):
            raise ValueError(name)

    def get(self, name: str) -> np.ndarray:
        a = np.empty(self.shape(name))
        if self._lib.oc_get_field(self._p, FIELDS[name], _ptr(a)):
            raise ValueError(name)
        return a

    def step(self, nsteps: int = 1):
        rc = self._lib.oc_step(self._p, nsteps)
        if rc:
            raise RuntimeError(f"oc_step failed ({rc})")

    def half_step_e(self, r_signed: float):
        if self._lib.oc_half_step_e(self._p, r_signed):
            raise RuntimeError("oc_half_step_e")

    def half_step_h(self, r_signed: float):
        if self._lib.oc_half_step_h(self._p, r_signed):
            raise RuntimeError("oc_half_step_h")

    def cg_stats(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        self._lib.oc_cg_stats(self._p, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def apply_m(self, name: str, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.shape(name))
        y = np.empty_like(x)
        if self._lib.oc_apply_m(self._p, FIELDS[name], _ptr(x), _ptr(y)):
            raise ValueError(name)
        return y

    def solve_m(self, name: str, b) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(self.shape(name))
        x = np.empty_like(b)
        it = self._lib.oc_solve_m(self._p, FIELDS[name], _ptr(b), _ptr(x))
        if it < 0:
            raise ValueError(name)
        return x

    def init_h_taylor(self):
        """Replace H (at tau = 0) by H at tau = h_tau/2 (eq:talorh)."""
        if self._lib.oc_init_h_taylor(self._p):
            raise RuntimeError("oc_init_h_taylor")

    def rhs(self, name: str) -> np.ndarray:
        out = np.empty(self.shape(name))
        if self._lib.oc_rhs(self._p, FIELDS[name], _ptr(out)):
            raise ValueError(name)
        return out
