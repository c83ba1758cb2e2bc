"""Python handle over a c4m batch: many independent 2D problems of uneven N
advanced together (one persistent launch per phase, a HIP graph per step)."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .problem import Problem, make_config


class Batch:
    def __init__(self, specs, *, device="cuda", stream=None, **common):
        """specs: list of dicts with at least `n` (and optionally `cfl`);
        `common` holds the keyword settings shared by every problem."""
        self._lib = L.load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.specs = [dict(s) for s in specs]
        cfgs = (L.C4mConfig * len(specs))()
        for i, s in enumerate(self.specs):
            cfgs[i] = make_config(2, s["n"], s.get("cfl", 0.5), **common)
        self._cfgs = cfgs
        nb = ctypes.c_size_t()
        L.check(self._lib.c4m_batch_workspace_bytes(cfgs, len(specs), ctypes.byref(nb)),
                "c4m_batch_workspace_bytes")
        self.nbytes = nb.value
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        L.check(self._lib.c4m_batch_create(cfgs, len(specs), ctypes.c_void_p(self.workspace.data_ptr()),
                                           self.nbytes, ctypes.c_void_p(int(self.stream.cuda_stream)),
                                           ctypes.byref(self._h)), "c4m_batch_create")
        self.problems = []
        for i, s in enumerate(self.specs):
            ph = ctypes.c_void_p()
            L.check(self._lib.c4m_batch_problem(self._h, i, ctypes.byref(ph)), "c4m_batch_problem")
            self.problems.append(Problem(2, s["n"], s.get("cfl", 0.5), device=device, stream=self.stream,
                                         _borrowed=ph, **common))

    @classmethod
    def from_problems(cls, problems, *, stream=None):
        """A batch over existing 2D problems (their fields stay where they
        are); only the work-queue tables are allocated."""
        self = cls.__new__(cls)
        self._lib = L.load()
        self.problems = list(problems)
        self.device = problems[0].device
        self.stream = stream if stream is not None else problems[0].stream
        self.specs = [{"n": p.n, "cfl": p.cfl} for p in problems]
        nb = ctypes.c_size_t()
        arr = (ctypes.c_void_p * len(problems))(*[p.handle.value for p in problems])
        L.check(self._lib.c4m_batch_tables_bytes(arr, len(problems), ctypes.byref(nb)), "c4m_batch_tables_bytes")
        self.nbytes = nb.value
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        L.check(self._lib.c4m_batch_create_from(arr, len(problems), ctypes.c_void_p(self.workspace.data_ptr()),
                                                self.nbytes, ctypes.c_void_p(int(self.stream.cuda_stream)),
                                                ctypes.byref(self._h)), "c4m_batch_create_from")
        self._borrowed_problems = True
        return self

    def __len__(self):
        return len(self.problems)

    def __getitem__(self, i) -> Problem:
        return self.problems[i]

    def step(self, nsteps: int = 1):
        L.check(self._lib.c4m_batch_step(self._h, int(nsteps)), "c4m_batch_step")

    def info(self) -> dict:
        """Summed member figures and, when profiling, kernel time per class."""
        inf = L.C4mInfo()
        L.check(self._lib.c4m_batch_get_info(self._h, ctypes.byref(inf)), "c4m_batch_get_info")
        out = {}
        for f, _ in L.C4mInfo._fields_:
            v = getattr(inf, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out

    def check(self):
        """Synchronise; raise if a stage wait of an earlier step gave up."""
        L.check(self._lib.c4m_batch_check(self._h), "c4m_batch_check")

    def close(self):
        if self._h:
            if not getattr(self, "_borrowed_problems", False):
                for p in self.problems:
                    p.close()
            L.check(self._lib.c4m_batch_destroy(self._h), "c4m_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
