"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/c4m.h declares, and rejects bad configurations before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2306_17263_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libc4m.so not built (run __graft_entry__.build())")
    return L, L.load()


def test_header_declarations_are_exported():
    L, lib = _lib()
    header = open(os.path.join(ROOT, "include", "c4m.h")).read()
    declared = set(re.findall(r"\b(c4m_[a-z_]+)\s*\(", header))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_config_validation_without_device():
    from paper_2306_17263_amd.problem import make_config
    L, lib = _lib()
    out = ctypes.c_size_t()
    cfg = make_config(dim=2, n=64)
    assert lib.c4m_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == L.OK
    assert out.value > 4 * 65 * 80 * 8
    bad = make_config(dim=2, n=4)
    assert lib.c4m_workspace_bytes(ctypes.byref(bad), ctypes.byref(out)) == L.EINVAL
    unstable = make_config(dim=2, n=64, cfl=0.70)
    assert lib.c4m_workspace_bytes(ctypes.byref(unstable), ctypes.byref(out)) == L.EUNSTABLE
    assert b"stability" in lib.c4m_last_error()
    forced = make_config(dim=2, n=64, cfl=0.70, flags=L.FLAG_ALLOW_ANY_CFL)
    assert lib.c4m_workspace_bytes(ctypes.byref(forced), ctypes.byref(out)) == L.OK
    cfg3 = make_config(dim=3, n=32, cfl=0.5)
    assert lib.c4m_workspace_bytes(ctypes.byref(cfg3), ctypes.byref(out)) == L.EUNSTABLE
    # the PCG form takes more temporaries; it runs in FP64 only
    pcg = make_config(dim=2, n=64, solver="pcg")
    pb = ctypes.c_size_t()
    assert lib.c4m_workspace_bytes(ctypes.byref(pcg), ctypes.byref(pb)) == L.OK
    assert pb.value > out.value
    pcg32 = make_config(dim=2, n=64, solver="pcg", precision="fp32_refined")
    assert lib.c4m_workspace_bytes(ctypes.byref(pcg32), ctypes.byref(pb)) == L.EINVAL
    bad_iter = make_config(dim=2, n=64, solver="pcg", max_iter=-1)
    assert lib.c4m_workspace_bytes(ctypes.byref(bad_iter), ctypes.byref(pb)) == L.EINVAL
    # create rejects a misaligned or small workspace before any device call
    h = ctypes.c_void_p()
    assert lib.c4m_create(ctypes.byref(cfg), ctypes.c_void_p(16), 1 << 30, None, ctypes.byref(h)) == L.EINVAL
    assert lib.c4m_create(ctypes.byref(cfg), ctypes.c_void_p(4096), 16, None, ctypes.byref(h)) == L.ENOMEM


def test_status_strings():
    L, lib = _lib()
    for s in range(0, -8, -1):
        assert lib.c4m_status_string(s)


def test_source_entry_points_without_device():
    """c4m_source_work_bytes / c4m_step_source reject a missing problem or
    source before any device call; the ctypes struct matches the header's
    member list."""
    L, lib = _lib()
    assert lib.c4m_source_work_bytes(None) == 0
    src = L.C4mSourceTM()
    assert lib.c4m_step_source(None, ctypes.byref(src), None, 0) == L.EINVAL
    header = open(os.path.join(ROOT, "include", "c4m.h")).read()
    body = header[header.index("typedef struct c4m_source_tm {"):header.index("} c4m_source_tm;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    members = re.findall(r"\b(\w+)(?:\[2\]\[2\])?;", body)
    assert members == [f[0] for f in L.C4mSourceTM._fields_]
