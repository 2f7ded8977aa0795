"""Shearing-box Poisson solver for AMD MI355X: thin Python binding over the C ABI (include/sbp.h).

The binding only marshals arguments: every step of a solve runs in the HIP library.
PyTorch supplies device memory and the stream.  If the library is not built, creating a
plan raises; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import json
from dataclasses import dataclass
from typing import Optional, Sequence, Union

from . import _lib
from ._lib import (SBP_FLAG_AUTOTUNE, SBP_FLAG_FIVE_PASS, SBP_FLAG_FUSED, SBP_FLAG_GRAPH, SBP_FLAG_PLAIN, SbpBox,
                   SbpShear)

__all__ = ["Box", "Shear", "Plan", "SbpError", "load_library"]


class SbpError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        self.name = _lib.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{what}: {self.name}: {_detail()}")


def _detail() -> str:
    lib = _lib.load()
    msg = lib.sbp_last_error()
    return msg.decode() if msg else ""


def load_library():
    return _lib.load()


@dataclass(frozen=True)
class Box:
    """Geometry and method of one box (see sbp_box in include/sbp.h)."""

    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    pad: int = 2
    alpha: float = 0.0
    method: str = "vgf"  # "vgf" or "sasha"
    remap: str = "spectral"  # map to the periodic frame: "spectral" or "linear" (interpolation)

    def to_c(self) -> SbpBox:
        m = {"vgf": _lib.SBP_VGF, "sasha": _lib.SBP_SASHA}.get(self.method, -1)
        r = {"spectral": _lib.SBP_REMAP_SPECTRAL, "linear": _lib.SBP_REMAP_LINEAR}.get(self.remap, -1)
        return SbpBox(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, self.pad, self.alpha, m, r)


@dataclass(frozen=True)
class Shear:
    """Per-solve parameters: shear rate q, rotation rate Omega, time t, gravitational constant G."""

    q: float = 1.5
    omega: float = 1.0
    t: float = 0.0
    G: float = 1.0


def _check(status: int, what: str):
    if status != _lib.SBP_OK:
        raise SbpError(status, what)


class Plan:
    """A solve plan for one or more boxes (sbp_plan_create ... sbp_plan_destroy)."""

    def __init__(self, boxes: Union[Box, Sequence[Box]], precision: str = "fp32", device: int = 0,
                 graph: bool = False, autotune: bool = False, plain: bool = False, schedule: str = "auto"):
        self._lib = _lib.load()
        self.boxes = [boxes] if isinstance(boxes, Box) else list(boxes)
        self.precision = precision
        prec = {"fp64": _lib.SBP_FP64, "fp32": _lib.SBP_FP32}.get(precision, -1)
        flags = ((SBP_FLAG_GRAPH if graph else 0) | (SBP_FLAG_AUTOTUNE if autotune else 0)
                 | (SBP_FLAG_PLAIN if plain else 0)
                 | {"auto": 0, "fused": SBP_FLAG_FUSED, "five_pass": SBP_FLAG_FIVE_PASS}.get(schedule, 0x8000))
        arr = (SbpBox * len(self.boxes))(*[b.to_c() for b in self.boxes])
        h = ctypes.c_void_p()
        self._h = None
        _check(self._lib.sbp_plan_create(arr, len(self.boxes), prec, device, flags, ctypes.byref(h)), "sbp_plan_create")
        self._h = h
        self.device = device
        self._ws = None

    # -- workspace -------------------------------------------------------------------------
    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(self._lib.sbp_workspace_size(self._h, ctypes.byref(n)), "sbp_workspace_size")
        return n.value

    def set_workspace(self, tensor) -> None:
        """Hand the plan a caller-owned device buffer (a torch tensor) or None."""
        if tensor is None:
            _check(self._lib.sbp_set_workspace(self._h, None, 0), "sbp_set_workspace")
            self._ws = None
            return
        nbytes = tensor.numel() * tensor.element_size()
        _check(self._lib.sbp_set_workspace(self._h, ctypes.c_void_p(tensor.data_ptr()), nbytes), "sbp_set_workspace")
        self._ws = tensor

    # -- solve -----------------------------------------------------------------------------
    def solve(self, rho, phi, shear: Union[Shear, Sequence[Shear]], stream=None) -> None:
        """Enqueue one solve: rho, phi are device tensors (or lists, one per box) of shape
        (nx, ny, nz), C-contiguous, float32 for fp32 plans and float64 for fp64 plans."""
        self._solve(self._lib.sbp_solve, "sbp_solve", rho, phi, shear, stream)

    def solve_static(self, rho, phi, shear: Union[Shear, Sequence[Shear]], stream=None) -> None:
        """As solve, through sbp_solve_static: the workspace is the library's fixed per-device
        array, so the call allocates nothing (see include/sbp.h for its limits)."""
        self._solve(self._lib.sbp_solve_static, "sbp_solve_static", rho, phi, shear, stream)

    def _solve(self, fn, what, rho, phi, shear, stream) -> None:
        import torch

        rhos = [rho] if not isinstance(rho, (list, tuple)) else list(rho)
        phis = [phi] if not isinstance(phi, (list, tuple)) else list(phi)
        shears = [shear] if isinstance(shear, Shear) else list(shear)
        nb = len(self.boxes)
        if not (len(rhos) == len(phis) == len(shears) == nb):
            raise ValueError(f"expected {nb} rho/phi/shear entries")
        dt = torch.float32 if self.precision == "fp32" else torch.float64
        for b, (r, p) in enumerate(zip(rhos, phis)):
            shape = (self.boxes[b].nx, self.boxes[b].ny, self.boxes[b].nz)
            for name, t in (("rho", r), ("phi", p)):
                if not t.is_cuda or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
                    raise ValueError(f"box {b}: {name} must be a contiguous {dt} CUDA tensor of shape {shape}")
        rp = (ctypes.c_void_p * nb)(*[r.data_ptr() for r in rhos])
        pp = (ctypes.c_void_p * nb)(*[p.data_ptr() for p in phis])
        sp = (SbpShear * nb)(*[SbpShear(s.q, s.omega, s.t, s.G) for s in shears])
        if stream is None:
            stream = torch.cuda.current_stream(rhos[0].device)
        st = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(fn(self._h, rp, pp, sp, ctypes.c_void_p(st)), what)

    # -- output for the hydrodynamics ------------------------------------------------------
    def _check_tensors(self, groups, shapes):
        import torch

        dt = torch.float32 if self.precision == "fp32" else torch.float64
        for name, ts in groups:
            for b, t in enumerate(ts):
                if not t.is_cuda or t.dtype != dt or tuple(t.shape) != shapes[b] or not t.is_contiguous():
                    raise ValueError(f"box {b}: {name} must be a contiguous {dt} CUDA tensor of shape {shapes[b]}")

    @staticmethod
    def _stream(stream, t):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(t.device)
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)

    def ghosts(self, phi, out, ng: int, stream=None) -> None:
        """Potential with ng vertical ghost layers (sbp_ghosts): out has shape (nx, ny, nz + 2 ng)."""
        phis = [phi] if not isinstance(phi, (list, tuple)) else list(phi)
        outs = [out] if not isinstance(out, (list, tuple)) else list(out)
        nb = len(self.boxes)
        if not (len(phis) == len(outs) == nb):
            raise ValueError(f"expected {nb} phi/out entries")
        self._check_tensors([("phi", phis)], [(b.nx, b.ny, b.nz) for b in self.boxes])
        self._check_tensors([("out", outs)], [(b.nx, b.ny, b.nz + 2 * ng) for b in self.boxes])
        pp = (ctypes.c_void_p * nb)(*[p.data_ptr() for p in phis])
        op = (ctypes.c_void_p * nb)(*[o.data_ptr() for o in outs])
        _check(self._lib.sbp_ghosts(self._h, pp, op, ng, ctypes.c_void_p(self._stream(stream, phis[0]))),
               "sbp_ghosts")

    def gravity(self, phi, gx, gy, gz, shear: Union[Shear, Sequence[Shear]], stream=None) -> None:
        """Acceleration -grad Phi (sbp_gravity) into gx, gy, gz, each shaped like phi."""
        lists = [[v] if not isinstance(v, (list, tuple)) else list(v) for v in (phi, gx, gy, gz)]
        shears = [shear] if isinstance(shear, Shear) else list(shear)
        nb = len(self.boxes)
        if any(len(v) != nb for v in lists) or len(shears) != nb:
            raise ValueError(f"expected {nb} entries per argument")
        shapes = [(b.nx, b.ny, b.nz) for b in self.boxes]
        self._check_tensors(list(zip(("phi", "gx", "gy", "gz"), lists)), shapes)
        arrs = [(ctypes.c_void_p * nb)(*[t.data_ptr() for t in v]) for v in lists]
        sp = (SbpShear * nb)(*[SbpShear(s.q, s.omega, s.t, s.G) for s in shears])
        _check(self._lib.sbp_gravity(self._h, *arrs, sp, ctypes.c_void_p(self._stream(stream, lists[0][0]))),
               "sbp_gravity")

    # -- instrumentation -------------------------------------------------------------------
    def profile_enable(self, on: bool = True) -> None:
        _check(self._lib.sbp_profile_enable(self._h, 1 if on else 0), "sbp_profile_enable")

    def profile_read(self) -> dict:
        """{kernel name: (launches, total ms)} since the last read (synchronises the events)."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        launches = (ctypes.c_int64 * cap)()
        total = (ctypes.c_double * cap)()
        cnt = ctypes.c_int32()
        _check(self._lib.sbp_profile_read(self._h, names, launches, total, cap, ctypes.byref(cnt)), "sbp_profile_read")
        return {names[i].decode(): (launches[i], total[i]) for i in range(min(cnt.value, cap))}

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(4096)
        _check(self._lib.sbp_plan_describe(self._h, buf, len(buf)), "sbp_plan_describe")
        return json.loads(buf.value.decode())

    # -- lifetime --------------------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.sbp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
