"""ctypes declarations of the C ABI in include/c4m.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libc4m.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOCONV, EUNSTABLE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
FIELD = {"ex": 0, "ey": 1, "ez": 2, "hx": 3, "hy": 4, "hz": 5, "lx": 6, "ly": 7, "lz": 8}
CLOSURE = {"paper": 0, "reflect": 1}
LAP = {"tracked": 0, "discrete": 1}
PRECISION = {"fp64": 0, "fp32_refined": 1}
SOLVER = {"chebyshev": 0, "pcg": 1, "transform": 2}
SCHEME = {"c4": 0, "nc": 1}
FLAG_ALLOW_ANY_CFL = 0x1
FLAG_CHECK_FINITE = 0x2
FLAG_PROFILE = 0x4
FLAG_DIRECT = 0x8
KERNEL_CLASSES = ["rhs_e", "solve_e", "rhs_h", "solve_h", "step_e", "step_h", "other", "step"]

# every symbol include/c4m.h declares
EXPORTS = [
    "c4m_config_default", "c4m_workspace_bytes", "c4m_create", "c4m_field_shape",
    "c4m_set_field", "c4m_set_boundary", "c4m_get_field", "c4m_step", "c4m_init_h_taylor", "c4m_prepare",
    "c4m_set_stream", "c4m_get_info", "c4m_destroy",
    "c4m_batch_workspace_bytes", "c4m_batch_create", "c4m_batch_problem", "c4m_batch_step",
    "c4m_batch_check", "c4m_batch_get_info", "c4m_batch_destroy", "c4m_batch_tables_bytes", "c4m_batch_create_from",
    "c4m_step_fields_noalloc", "c4m_source_work_bytes", "c4m_step_source", "c4m_status_string", "c4m_last_error",
]


_Wall = (ctypes.c_void_p * 2) * 2


class C4mSourceTM(ctypes.Structure):
    """c4m_source_tm: device pointers of one sourced 2D step (NULL = zeros)."""
    _fields_ = [("jz", ctypes.c_void_p), ("jz_tt", ctypes.c_void_p), ("jz_lap", ctypes.c_void_p),
                ("jz_tt_lap", ctypes.c_void_p), ("hx_wall", _Wall), ("hy_wall", _Wall),
                ("jz_t", ctypes.c_void_p), ("kx", ctypes.c_void_p), ("kx_lap", ctypes.c_void_p),
                ("ky", ctypes.c_void_p), ("ky_lap", ctypes.c_void_p), ("dhx_wall", _Wall), ("dhy_wall", _Wall)]


class C4mConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("cfl", ctypes.c_double),
        ("z", ctypes.c_double), ("closure", ctypes.c_int32), ("lap_mode", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("solver", ctypes.c_int32), ("sweeps", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double), ("tile_x", ctypes.c_int32),
        ("tile_y", ctypes.c_int32), ("flags", ctypes.c_uint32), ("batch_wait_limit", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
    ]


class C4mInfo(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("tau_e", ctypes.c_double), ("tau_h", ctypes.c_double),
        ("sweeps", ctypes.c_int32), ("last_iters", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("last_rel_residual", ctypes.c_double), ("nonfinite", ctypes.c_int32),
        ("noconv", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t),
        ("kernel_ms", ctypes.c_double * 8), ("kernel_launches", ctypes.c_int64 * 8),
        ("kernel_alg_bytes", ctypes.c_double * 8),
    ]


class C4mError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load():
    """Load libc4m.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2306_17263_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cfgp = ctypes.POINTER(C4mConfig)
    lib.c4m_config_default.argtypes = [cfgp]
    lib.c4m_workspace_bytes.argtypes = [cfgp, ctypes.POINTER(sz)]
    lib.c4m_create.argtypes = [cfgp, vp, sz, vp, ctypes.POINTER(vp)]
    lib.c4m_field_shape.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.c4m_set_field.argtypes = [vp, i32, vp, i32]
    lib.c4m_set_boundary.argtypes = [vp, i32, i32, vp, i32]
    lib.c4m_get_field.argtypes = [vp, i32, vp, i32]
    lib.c4m_step.argtypes = [vp, i64]
    lib.c4m_init_h_taylor.argtypes = [vp]
    lib.c4m_prepare.argtypes = [vp, i64]
    lib.c4m_set_stream.argtypes = [vp, vp]
    lib.c4m_get_info.argtypes = [vp, ctypes.POINTER(C4mInfo)]
    lib.c4m_destroy.argtypes = [vp]
    lib.c4m_batch_workspace_bytes.argtypes = [cfgp, i32, ctypes.POINTER(sz)]
    lib.c4m_batch_create.argtypes = [cfgp, i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.c4m_batch_problem.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.c4m_batch_step.argtypes = [vp, i64]
    lib.c4m_batch_check.argtypes = [vp]
    lib.c4m_batch_get_info.argtypes = [vp, ctypes.POINTER(C4mInfo)]
    lib.c4m_batch_destroy.argtypes = [vp]
    lib.c4m_batch_tables_bytes.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(sz)]
    lib.c4m_batch_create_from.argtypes = [ctypes.POINTER(vp), i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.c4m_step_fields_noalloc.argtypes = [cfgp, ctypes.POINTER(vp), i64, vp]
    lib.c4m_source_work_bytes.argtypes = [vp]
    lib.c4m_source_work_bytes.restype = sz
    lib.c4m_step_source.argtypes = [vp, ctypes.POINTER(C4mSourceTM), vp, sz]
    for name in EXPORTS:
        if name in ("c4m_status_string", "c4m_last_error", "c4m_source_work_bytes"):
            continue
        getattr(lib, name).restype = ctypes.c_int
    lib.c4m_status_string.argtypes = [ctypes.c_int]
    lib.c4m_status_string.restype = ctypes.c_char_p
    lib.c4m_last_error.argtypes = []
    lib.c4m_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != OK:
        lib = load()
        detail = (lib.c4m_last_error() or b"").decode() or lib.c4m_status_string(status).decode()
        raise C4mError(status, where, detail)
