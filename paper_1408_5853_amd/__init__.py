"""cryocell: the explicit-implicit heat-conduction stepper of arXiv 1408.5853
on one MI355X, behind the C ABI of include/cryocell.h.

This module is argument marshalling over the HIP library: PyTorch supplies
device memory and the current stream; every step of the method runs in the
library's gfx950 kernels.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import CryoError, check, lib

__all__ = ["Plan", "CryoError", "validate", "stability_dt_max", "version"]


def version():
    return lib().cryo_version().decode()


def validate(cell):
    ps = _abi.ProblemStruct(cell)
    check(lib().cryo_validate(ps.ref()))


def stability_dt_max(cell, T_min):
    ps = _abi.ProblemStruct(cell)
    out = C.c_double()
    check(lib().cryo_stability_dt_max(ps.ref(), float(T_min), C.byref(out)))
    return out.value


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Plan:
    """A solver plan for one cell (problem dictionary, see cellgen)."""

    def __init__(self, cell, dtype="f64"):
        self.cell = cell
        self.dtype = dtype
        self._ps = _abi.ProblemStruct(cell)
        h = C.c_void_p()
        check(lib().cryo_plan_create(self._ps.ref(), _abi.F64 if dtype == "f64" else _abi.F32,
                                     C.byref(h)))
        self._h = h
        self.nr, self.nz = int(cell["nr"]), int(cell["nz"])

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().cryo_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.dtype == "f64" else torch.float32

    def radii(self):
        r = np.zeros(self.nr)
        check(lib().cryo_grid_radii(self._h, r.ctypes.data_as(C.POINTER(C.c_double))))
        return r

    def source_fraction(self, k0, n):
        s = np.zeros(int(n))
        check(lib().cryo_source_fraction(self._h, int(k0), int(n),
                                         s.ctypes.data_as(C.POINTER(C.c_double))))
        return s

    def workspace_bytes(self, nsteps):
        b = C.c_size_t()
        check(lib().cryo_workspace_bytes(self._h, int(nsteps), C.byref(b)))
        return b.value

    def workspace(self, nsteps, device="cuda"):
        torch = _torch()
        ws = torch.empty(self.workspace_bytes(nsteps), dtype=torch.uint8, device=device)
        assert ws.data_ptr() % 256 == 0
        return ws

    @property
    def field_shape(self):
        """(nz, nr) for f64; (2, nz, nr) for f32 (value plane, residual plane)."""
        return (self.nz, self.nr) if self.dtype == "f64" else (2, self.nz, self.nr)

    def init(self, T=None, stream=None):
        torch = _torch()
        if T is None:
            T = torch.empty(self.field_shape, dtype=self.torch_dtype, device="cuda")
        self._check_field(T)
        check(lib().cryo_init(self._h, _ptr(T), _stream(stream)))
        return T

    def field_from(self, T0):
        """A device field holding the float64 array T0 [nz][nr]."""
        torch = _torch()
        T0 = torch.as_tensor(np.asarray(T0, dtype=np.float64))
        if self.dtype == "f64":
            return T0.to("cuda").contiguous()
        hi = T0.to(torch.float32)
        lo = (T0 - hi.to(torch.float64)).to(torch.float32)
        return torch.stack([hi, lo]).to("cuda").contiguous()

    @staticmethod
    def field_values(T):
        """float64 host array [nz][nr] of a device field (f32 pairs summed)."""
        t = T.detach().to("cpu").to(_torch().float64)
        return (t if t.dim() == 2 else t[0] + t[1]).numpy()

    def _check_field(self, T):
        if tuple(T.shape) != self.field_shape or T.dtype != self.torch_dtype or not T.is_cuda \
                or not T.is_contiguous():
            raise ValueError("field must be a contiguous %s CUDA tensor of shape %s"
                             % (self.torch_dtype, self.field_shape))

    def forward(self, T, k0=0, nsteps=None, ws=None, surf=None, stream=None):
        """Advance T in place by nsteps steps from global step k0.  `surf`, if
        given, is a float64 CUDA tensor of length >= nsteps for the surface
        mean after each step.  Asynchronous on the stream."""
        n = int(self.cell["nsteps"] if nsteps is None else nsteps)
        self._check_field(T)
        if ws is None:
            ws = self.workspace(n, T.device)
        sp = None
        if surf is not None:
            torch = _torch()
            if surf.dtype != torch.float64 or not surf.is_cuda or surf.numel() < n:
                raise ValueError("surf must be a float64 CUDA tensor of length >= nsteps")
            sp = _ptr(surf)
        check(lib().cryo_forward(self._h, _ptr(T), int(k0), n, _ptr(ws), ws.numel(), sp,
                                 _stream(stream)))
        return T

    def poll(self, ws, stream=None):
        check(lib().cryo_poll(self._h, _ptr(ws), _stream(stream)))
