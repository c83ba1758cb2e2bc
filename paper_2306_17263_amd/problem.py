"""Python handle over one c4m problem.  PyTorch supplies the device workspace
and the HIP stream; every step of the scheme runs in libc4m.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from contextlib import nullcontext as _nullctx


def make_config(dim: int = 2, n: int = 64, cfl: float = 0.5, z: float = 1.0,
                closure: str = "paper", lap_mode: str = "tracked", precision: str = "fp64",
                solver: str = "chebyshev", sweeps: int = 0, max_iter: int = 0, rtol: float = 0.0,
                tile_x: int = 0, tile_y: int = 0, flags: int = 0,
                batch_wait_limit: int = 0, scheme: str = "c4") -> L.C4mConfig:
    lib = L.load()
    cfg = L.C4mConfig()
    L.check(lib.c4m_config_default(ctypes.byref(cfg)), "c4m_config_default")
    cfg.dim, cfg.n, cfg.cfl, cfg.z = dim, n, cfl, z
    cfg.closure = L.CLOSURE[closure]
    cfg.lap_mode = L.LAP[lap_mode]
    cfg.precision = L.PRECISION[precision]
    cfg.solver = L.SOLVER[solver]
    cfg.sweeps, cfg.max_iter, cfg.rtol = sweeps, max_iter, rtol
    cfg.tile_x, cfg.tile_y, cfg.flags = tile_x, tile_y, flags
    cfg.batch_wait_limit = batch_wait_limit
    cfg.scheme = L.SCHEME[scheme]
    return cfg


def workspace_bytes(cfg: L.C4mConfig) -> int:
    lib = L.load()
    out = ctypes.c_size_t()
    L.check(lib.c4m_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "c4m_workspace_bytes")
    return out.value


def _stream_ptr(stream) -> int:
    return int(stream.cuda_stream)


class Problem:
    """One PEC cavity problem resident on the device."""

    def __init__(self, dim: int = 2, n: int = 64, cfl: float = 0.5, *, device="cuda",
                 stream=None, _borrowed=None, **kw):
        self._lib = L.load()
        self.cfg = make_config(dim, n, cfl, **kw)
        self._owned = _borrowed is None
        if _borrowed is not None:             # a member of a Batch: handle owned by the batch
            self.device = torch.device(device)
            self.stream = stream
            self._h = _borrowed
            self.dim, self.n, self.cfl = dim, n, cfl
            return
        self.device = torch.device(device)
        self.nbytes = workspace_bytes(self.cfg)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        L.check(self._lib.c4m_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                                     self.nbytes, ctypes.c_void_p(_stream_ptr(self.stream)),
                                     ctypes.byref(self._h)), "c4m_create")
        self.dim, self.n, self.cfl = dim, n, cfl

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._owned:
            L.check(self._lib.c4m_destroy(self._h), "c4m_destroy")
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, name: str):
        s = (ctypes.c_int64 * 3)()
        L.check(self._lib.c4m_field_shape(self._h, L.FIELD[name], s), f"c4m_field_shape({name})")
        return (s[0], s[1], s[2])

    def set(self, name: str, value):
        shp = self.shape(name)
        if isinstance(value, torch.Tensor) and value.is_cuda:
            t = value.to(torch.float64).contiguous().reshape(shp)
            self._keep = t
            L.check(self._lib.c4m_set_field(self._h, L.FIELD[name], ctypes.c_void_p(t.data_ptr()), 1),
                    f"c4m_set_field({name})")
            return
        a = np.ascontiguousarray(np.asarray(value, dtype=np.float64).reshape(shp))
        L.check(self._lib.c4m_set_field(self._h, L.FIELD[name], a.ctypes.data_as(ctypes.c_void_p), 0),
                f"c4m_set_field({name})")

    def set_boundary(self, name: str, face: int, values):
        """Wall plane of one component on face 2 axis + side (c4m_set_boundary)."""
        shp = list(self.shape(name))
        axis = face // 2
        del shp[2 - axis]
        if isinstance(values, torch.Tensor) and values.is_cuda:
            t = values.to(torch.float64).contiguous().reshape(shp)
            self._keep = t
            L.check(self._lib.c4m_set_boundary(self._h, L.FIELD[name], int(face), ctypes.c_void_p(t.data_ptr()), 1),
                    f"c4m_set_boundary({name}, {face})")
            return
        a = np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(shp))
        L.check(self._lib.c4m_set_boundary(self._h, L.FIELD[name], int(face), a.ctypes.data_as(ctypes.c_void_p), 0),
                f"c4m_set_boundary({name}, {face})")

    def get(self, name: str, device: bool = False):
        shp = self.shape(name)
        if device:
            out = torch.empty(shp, dtype=torch.float64, device=self.device)
            L.check(self._lib.c4m_get_field(self._h, L.FIELD[name], ctypes.c_void_p(out.data_ptr()), 1),
                    f"c4m_get_field({name})")
            return out
        out = np.empty(shp, dtype=np.float64)
        L.check(self._lib.c4m_get_field(self._h, L.FIELD[name], out.ctypes.data_as(ctypes.c_void_p), 0),
                f"c4m_get_field({name})")
        return out

    def init_h_taylor(self):
        """Replace H (set at tau = 0) by H at tau = h_tau/2 (Taylor start)."""
        L.check(self._lib.c4m_init_h_taylor(self._h), "c4m_init_h_taylor")

    SOURCE_ARRAYS = ("jz", "jz_tt", "jz_lap", "jz_tt_lap", "jz_t", "kx", "kx_lap", "ky", "ky_lap")
    SOURCE_WALLS = ("hx_wall", "hy_wall", "dhx_wall", "dhy_wall")

    def step_source(self, data: dict):
        """One step with a current J = (0, 0, Jz) (2D, compact scheme, PAPER
        closure): `data` maps the member names of c4m_source_tm to arrays
        (numpy or CUDA tensors; a wall entry is [[first, third] at wall 0,
        [first, third] at wall 1]); a missing name stands for zeros.  The
        arrays are moved to the device on the problem's stream."""
        n = self.n
        shapes = {"kx": (n, n + 1), "kx_lap": (n, n + 1), "ky": (n + 1, n), "ky_lap": (n + 1, n)}
        keep = []
        src = L.C4mSourceTM()
        ctx = torch.cuda.stream(self.stream) if isinstance(self.stream, torch.cuda.Stream) else _nullctx()
        with ctx:
            def dev(a, shape):
                t = torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a)
                t = t.to(device=self.device, dtype=torch.float64).contiguous()
                if t.numel() != int(np.prod(shape)):
                    raise ValueError(f"source array of {t.numel()} values, expected shape {shape}")
                keep.append(t)
                return t.data_ptr()

            for name in self.SOURCE_ARRAYS:
                if data.get(name) is not None:
                    setattr(src, name, dev(data[name], shapes.get(name, (n + 1, n + 1))))
            for name in self.SOURCE_WALLS:
                walls = data.get(name)
                if walls is None:
                    continue
                slot = getattr(src, name)
                for w in (0, 1):
                    for d in (0, 1):
                        if walls[w][d] is not None:
                            slot[w][d] = dev(walls[w][d], (n + 1,))
            need = int(self._lib.c4m_source_work_bytes(self._h))
            if need == 0:
                raise L.C4mError(1, "c4m_step_source", "this problem takes no sources")
            if getattr(self, "_src_work", None) is None or self._src_work.numel() < need:
                self._src_work = torch.empty(need, dtype=torch.uint8, device=self.device)
        L.check(self._lib.c4m_step_source(self._h, ctypes.byref(src), ctypes.c_void_p(self._src_work.data_ptr()),
                                          need), "c4m_step_source")
        self._src_keep = keep   # released after the next call, stream-ordered

    def prepare(self, nsteps: int):
        """Capture the graphs that step(nsteps) replays, without running them."""
        L.check(self._lib.c4m_prepare(self._h, int(nsteps)), "c4m_prepare")

    def set_stream(self, stream):
        """Wait for the work queued on the current stream, then use `stream`."""
        L.check(self._lib.c4m_set_stream(self._h, ctypes.c_void_p(_stream_ptr(stream))), "c4m_set_stream")
        self.stream = stream

    def step(self, nsteps: int = 1):
        L.check(self._lib.c4m_step(self._h, int(nsteps)), "c4m_step")

    def info(self) -> dict:
        inf = L.C4mInfo()
        L.check(self._lib.c4m_get_info(self._h, ctypes.byref(inf)), "c4m_get_info")
        out = {}
        for f, _ in L.C4mInfo._fields_:
            v = getattr(inf, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out

    def fields(self):
        names = ["ez", "hx", "hy"] if self.dim == 2 else ["ex", "ey", "ez", "hx", "hy", "hz"]
        if self.cfg.lap_mode == L.LAP["tracked"] and self.cfg.scheme == L.SCHEME["c4"]:
            names += ["lz"] if self.dim == 2 else ["lx", "ly", "lz"]
        return names
