"""The no-allocation stepping call (c4m_step_fields_noalloc) against the
regular path (c4m_create on a caller workspace, set, step, get): the same
kernels on the same data, so the fields agree bit for bit.  Two calls in a
row, the second on a smaller grid (the static scratch keeps the first
call's contents; the call clears what must start at zero), then a 3D call,
and the size limit of the scratch."""
import ctypes

import numpy as np
import pytest

from gpu_util import random_fields

pytestmark = pytest.mark.gpu


def _noalloc(dim, n, r, init, steps, lap="tracked"):
    import torch
    from paper_2306_17263_amd import _lib as L
    from paper_2306_17263_amd.problem import make_config
    fn = L.load().c4m_step_fields_noalloc
    cfg = make_config(dim, n, r, lap_mode=lap)
    tens = {a: torch.from_numpy(np.ascontiguousarray(v)).cuda() for a, v in init.items()}
    ptrs = (ctypes.c_void_p * 9)()
    for a, t in tens.items():
        ptrs[L.FIELD[a]] = t.data_ptr()
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    L.check(fn(ctypes.byref(cfg), ptrs, steps, ctypes.c_void_p(st.cuda_stream)), "c4m_step_fields_noalloc")
    return {a: t.cpu().numpy() for a, t in tens.items()}


def _regular(dim, n, r, init, steps, lap="tracked"):
    from paper_2306_17263_amd import Problem
    p = Problem(dim, n, r, lap_mode=lap)
    for a, v in init.items():
        p.set(a, v)
    p.step(steps)
    out = {a: p.get(a) for a in init}
    p.close()
    return out


def _fields(dim, n, seed, lap):
    f = random_fields(dim, n, seed=seed)
    if lap != "tracked":
        f = {a: v for a, v in f.items() if a[0] != "l"}
    return f


@pytest.mark.parametrize("lap", ["tracked", "discrete"])
def test_noalloc_equals_regular_two_calls(lap):
    for dim, n, r, steps in ((2, 96, 0.5, 7), (2, 40, 0.5, 5), (3, 20, 0.4, 3)):
        init = _fields(dim, n, 100 + n, lap)
        got = _noalloc(dim, n, r, init, steps, lap)
        ref = _regular(dim, n, r, init, steps, lap)
        for a in init:
            assert np.array_equal(got[a], ref[a]), (dim, n, a)
        assert np.max(np.abs(got[[a for a in init if a[0] == "e"][0]] - init[[a for a in init if a[0] == "e"][0]])) > 0


def test_noalloc_rejects_sizes_beyond_scratch():
    from paper_2306_17263_amd import C4mError, ENOMEM
    init = _fields(2, 2048, 1, "discrete")
    with pytest.raises(C4mError) as ei:
        _noalloc(2, 2048, 0.5, init, 1, "discrete")
    assert ei.value.status == ENOMEM
