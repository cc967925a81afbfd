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

__all__ = ["Plan", "State", "Batch", "CryoError", "CryoSolve", "gradient", "gradient_plan",
           "with_params", "params_of", "autotune", "tune_batch",
           "validate", "stability_dt_max", "version"]


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
        if cell.get("poly"):
            Ls = cell["layers"]
            self.set_poly_laws([l["poly_a"] for l in Ls], [l["poly_b"] for l in Ls],
                               cell.get("joule_tref", 0.0))
        if cell.get("stepped"):
            self.set_stepped(cell["stepped"]["z_full"], cell["stepped"]["nr_top"])
        if cell.get("turn_on"):
            self.set_turn_on(True)

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

    def shape(self):
        """(rows per lane, waves per line, lines per wave) of the step kernel."""
        v = [C.c_int32() for _ in range(3)]
        check(lib().cryo_plan_shape(self._h, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_shape(self, rows_per_lane, waves_per_line, lines_per_wave):
        check(lib().cryo_plan_set_shape(self._h, int(rows_per_lane), int(waves_per_line),
                                        int(lines_per_wave)))

    def set_turn_on(self, on=True):
        """Switch the transient turn-on model of eq. (22) on or off: each
        pulse's first step then runs as 100 sub-steps of dt/100."""
        check(lib().cryo_plan_set_turn_on(self._h, int(bool(on))))

    def set_stepped(self, z_full, nr_top):
        """Stepped domain of eq. (9): lines above z_full span the inner nr_top
        radial nodes (the terminal); the surface mean covers lines 0..z_full."""
        check(lib().cryo_plan_set_stepped(self._h, int(z_full), int(nr_top)))

    def set_poly_laws(self, a, b, joule_tref=0.0):
        """Polynomial laws of eqs. (23), (24): a[m] = 4 capacity coefficients,
        b[m] = 5 conductivity coefficients per layer (ascending powers of T);
        joule_tref > 0 adds the T^(-1/2) Joule source of eq. (25)."""
        aa = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
        L = len(self.cell["layers"])
        if aa.size != 4 * L or bb.size != 5 * L:
            raise ValueError("need 4 capacity and 5 conductivity coefficients per layer")
        dp = C.POINTER(C.c_double)
        check(lib().cryo_plan_set_poly_laws(self._h, aa.ctypes.data_as(dp), bb.ctypes.data_as(dp),
                                            float(joule_tref)))

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

    def forward_noalloc(self, T, k0=0, nsteps=None, surf=None, stream=None):
        """As forward, with the workspace in the library's own device array
        (cryo_forward_noalloc: no allocation; the plan must have run once or
        have a State, so that its device tables exist)."""
        n = int(self.cell["nsteps"] if nsteps is None else nsteps)
        self._check_field(T)
        sp = None
        if surf is not None:
            torch = _torch()
            if surf.dtype != torch.float64 or not surf.is_cuda or surf.numel() < n:
                raise ValueError("surf must be a float64 CUDA tensor of length >= nsteps")
            sp = _ptr(surf)
        check(lib().cryo_forward_noalloc(self._h, _ptr(T), int(k0), n, sp, _stream(stream)))
        return T

    def poll(self, ws, stream=None):
        check(lib().cryo_poll(self._h, _ptr(ws), _stream(stream)))

    def _gradient_ready(self):
        if self.shape()[:2] not in _ADJOINT_SHAPES:
            # the adjoint kernels take 2, 4 or 8 rows per lane: switch to the
            # gradient shape while the plan has not run yet (else the library
            # reports the shape as unsupported)
            sh = _gradient_shape(self.cell)
            if sh is not None:
                try:
                    self.set_shape(*sh)
                except CryoError:
                    pass

    def gradient_workspace_bytes(self, nsteps, ckpt=0):
        b = C.c_size_t()
        check(lib().cryo_gradient_workspace_bytes(self._h, int(nsteps), int(ckpt), C.byref(b)))
        return b.value

    def set_gradient_store(self, steps):
        """Keep the states of the run's last `steps` kernel steps from the
        gradient's forward (cryo_plan_set_gradient_store): no recompute for
        them, one field of device memory each.  0: checkpoints only."""
        check(lib().cryo_plan_set_gradient_store(self._h, int(steps)))

    def gradient_store_for(self, nsteps, budget_bytes, ckpt=0):
        """The largest gradient store whose workspace for nsteps steps fits
        in budget_bytes (cryo_gradient_store_steps; 0 when none fits).  The
        plan's own setting is left as it is."""
        self._gradient_ready()
        d = C.c_int64()
        check(lib().cryo_gradient_store_steps(self._h, int(nsteps), int(ckpt),
                                              int(budget_bytes), C.byref(d)))
        return d.value

    def gradient(self, target, T0=None, nsteps=None, ckpt=0, stream=None, store=None):
        """J = sum_n (S_n - target_n)^2 and dJ/d[amplitude, width, thickness_m,
        k_scale_m] by the discrete adjoint (FP64 plans).  Returns (J, grad,
        surface trace) as float, numpy, numpy.  Synchronous.  `store` (when
        given) sets the plan's gradient store first."""
        torch = _torch()
        self._gradient_ready()
        if store is not None:
            self.set_gradient_store(store)
        n = int(self.cell["nsteps"] if nsteps is None else nsteps)
        tgt = np.ascontiguousarray(np.asarray(target, dtype=np.float64)[:n])
        if tgt.size < n:
            raise ValueError("target needs nsteps values")
        T = self.init() if T0 is None else self.field_from(T0)
        ws = torch.empty(self.gradient_workspace_bytes(n, ckpt), dtype=torch.uint8, device="cuda")
        J = C.c_double()
        L = len(self.cell["layers"])
        g = np.zeros(2 + 2 * L)
        S = np.zeros(n)
        dp = C.POINTER(C.c_double)
        check(lib().cryo_gradient(self._h, _ptr(T), n, tgt.ctypes.data_as(dp), int(ckpt),
                                  _ptr(ws), ws.numel(), C.byref(J), g.ctypes.data_as(dp),
                                  S.ctypes.data_as(dp), _stream(stream)))
        return J.value, g, S

    def gradient_async(self, target, T0, nsteps=None, ckpt=0, ws=None, stream=None, store=None):
        """The gradient enqueued on the stream with no host wait
        (cryo_gradient_async).  `target` (float64 CUDA tensor, nsteps values)
        and the field T0 (this plan's Field layout) are read on the device.
        Returns (J [1], grad [2 + 2L], surface trace [nsteps], ws), float64
        CUDA tensors and the workspace (made here when None), which must stay
        alive until the stream has finished; poll(ws) then reports a
        non-finite temperature.  `store` as for gradient."""
        torch = _torch()
        self._gradient_ready()
        if store is not None:
            self.set_gradient_store(store)
        n = int(self.cell["nsteps"] if nsteps is None else nsteps)
        if (target.dtype != torch.float64 or not target.is_cuda or target.numel() < n
                or not target.is_contiguous()):
            raise ValueError("target must be a contiguous float64 CUDA tensor of length >= nsteps")
        if ws is None:
            ws = torch.empty(self.gradient_workspace_bytes(n, ckpt), dtype=torch.uint8,
                             device="cuda")
        L = len(self.cell["layers"])
        J = torch.empty(1, dtype=torch.float64, device="cuda")
        g = torch.empty(2 + 2 * L, dtype=torch.float64, device="cuda")
        S = torch.empty(n, dtype=torch.float64, device="cuda")
        check(lib().cryo_gradient_async(self._h, _ptr(T0), n, _ptr(target),
                                        int(ckpt), _ptr(ws), ws.numel(), _ptr(J), _ptr(g),
                                        _ptr(S), _stream(stream)))
        return J, g, S, ws


class State:
    """A plan's field kept in the kernels' internal layout in device memory
    between calls (no layout conversion per call).  Calls on one State must
    go to one stream in order."""

    def __init__(self, plan, T=None, stream=None):
        torch = _torch()
        self.plan = plan
        self.mem = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device="cuda")
        assert self.mem.data_ptr() % 256 == 0
        h = C.c_void_p()
        check(lib().cryo_state_create(plan._h, _ptr(self.mem), self.mem.numel(), C.byref(h)))
        self._h = h
        if T is not None:
            self.load(T, stream)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().cryo_state_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, T, stream=None):
        self.plan._check_field(T)
        check(lib().cryo_state_load(self._h, _ptr(T), _stream(stream)))

    def forward(self, k0, nsteps, surf=None, stream=None):
        """nsteps steps from global step k0 (as Plan.forward)."""
        n = int(nsteps)
        sp = None
        if surf is not None:
            torch = _torch()
            if surf.dtype != torch.float64 or not surf.is_cuda or surf.numel() < n:
                raise ValueError("surf must be a float64 CUDA tensor of length >= nsteps")
            sp = _ptr(surf)
        check(lib().cryo_state_forward(self._h, int(k0), n, sp, _stream(stream)))

    def store(self, T=None, stream=None):
        torch = _torch()
        if T is None:
            T = torch.empty(self.plan.field_shape, dtype=self.plan.torch_dtype, device="cuda")
        self.plan._check_field(T)
        check(lib().cryo_state_store(self._h, _ptr(T), _stream(stream)))
        return T

    def poll(self, stream=None):
        self.plan.poll(self.mem, stream)


def _instance_options(cells):
    """Per-instance plan options of a batch: the polynomial laws (eqs.
    (23)-(25)) and the stepped domain (eq. (9)), as Plan takes them from a
    cell.  Returns the ctypes array and the arrays it points into (to be
    kept alive with it)."""
    n = len(cells)
    opts = (_abi.InstanceOptions * n)()
    keep = []
    dp = C.POINTER(C.c_double)
    for i, c in enumerate(cells):
        if c.get("poly"):
            Ls = c["layers"]
            a = np.ascontiguousarray([float(x) for l in Ls for x in l["poly_a"]])
            b = np.ascontiguousarray([float(x) for l in Ls for x in l["poly_b"]])
            keep += [a, b]
            opts[i].poly_a = a.ctypes.data_as(dp)
            opts[i].poly_b = b.ctypes.data_as(dp)
            opts[i].joule_tref = float(c.get("joule_tref", 0.0))
        if c.get("stepped"):
            opts[i].z_full = int(c["stepped"]["z_full"])
            opts[i].nr_top = int(c["stepped"]["nr_top"])
        opts[i].turn_on = int(bool(c.get("turn_on")))
    return opts, keep


class Batch:
    """Many independent cells stepped together (design sweeps)."""

    def __init__(self, cells, dtype="f64", shapes=None):
        self.cells = list(cells)
        self.dtype = dtype
        n = len(self.cells)
        self._ps = [_abi.ProblemStruct(c) for c in self.cells]
        arr = (_abi.Problem * n)(*[p.s for p in self._ps])
        self._arr = arr
        sh = None
        if shapes is not None:
            flat = np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(n, 3))
            self._shapes = flat
            sh = flat.ctypes.data_as(C.POINTER(C.c_int32))
        opts, self._keep = _instance_options(self.cells)
        h = C.c_void_p()
        check(lib().cryo_batch_create_with(n, arr, _abi.F64 if dtype == "f64" else _abi.F32, sh,
                                           opts, C.byref(h)))
        self._h = h
        off = (C.c_int64 * (n + 1))()
        check(lib().cryo_batch_offsets(self._h, off))
        self.offsets = [int(x) for x in off]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().cryo_batch_destroy(self._h)
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

    def shape(self, i):
        v = (C.c_int32 * 3)()
        check(lib().cryo_batch_shape(self._h, int(i), v))
        return tuple(v)

    def workspace(self, device="cuda"):
        torch = _torch()
        b = C.c_size_t()
        check(lib().cryo_batch_workspace_bytes(self._h, C.byref(b)))
        ws = torch.empty(b.value, dtype=torch.uint8, device=device)
        assert ws.data_ptr() % 256 == 0
        return ws

    def init(self, T=None, stream=None):
        torch = _torch()
        if T is None:
            T = torch.empty(self.offsets[-1], dtype=self.torch_dtype, device="cuda")
        check(lib().cryo_batch_init(self._h, _ptr(T), _stream(stream)))
        return T

    def field(self, T, i):
        """View of instance i's field in the packed buffer."""
        c = self.cells[i]
        v = T[self.offsets[i]:self.offsets[i + 1]]
        shp = (c["nz"], c["nr"]) if self.dtype == "f64" else (2, c["nz"], c["nr"])
        return v.view(shp)

    def forward(self, T, k0, nsteps, ws, stream=None):
        check(lib().cryo_batch_forward(self._h, _ptr(T), int(k0), int(nsteps), _ptr(ws),
                                       ws.numel(), _stream(stream)))
        return T

    def poll(self, ws, stream=None):
        bad = C.c_int32(-1)
        check(lib().cryo_batch_poll(self._h, _ptr(ws), _stream(stream), C.byref(bad)))


def autotune(cell, dtype="f64", steps=20, cache=None, stream=None):
    """Fastest (rows per lane, waves per line, lines per wave) for `cell`,
    timed on the GPU; returns (shape, us per step or -1 if cached)."""
    ps = _abi.ProblemStruct(cell)
    sh = (C.c_int32 * 3)()
    us = C.c_double()
    check(lib().cryo_autotune(ps.ref(), _abi.F64 if dtype == "f64" else _abi.F32, int(steps),
                              cache.encode() if cache else None, _stream(stream), sh,
                              C.byref(us)))
    return tuple(sh), us.value


def tune_batch(cells, dtype="f32", steps=64, cache=None, stream=None):
    """Per-instance launch shapes for Batch(cells, dtype, shapes=...), timed
    on the GPU per shape group (cryo_batch_autotune_with: cells may carry the
    polynomial laws, the stepped domain or the turn-on model, as Batch takes
    them); `cache` names an optional text file of earlier results."""
    n = len(cells)
    ps = [_abi.ProblemStruct(c) for c in cells]
    arr = (_abi.Problem * n)(*[p.s for p in ps])
    opts, keep = _instance_options(cells)
    out = (C.c_int32 * (3 * n))()
    check(lib().cryo_batch_autotune_with(n, arr, _abi.F64 if dtype == "f64" else _abi.F32,
                                         opts, int(steps), cache.encode() if cache else None,
                                         _stream(stream), out))
    del keep
    return [tuple(out[3 * i:3 * i + 3]) for i in range(n)]


def params_of(cell):
    """theta = [amplitude, width, thickness_0..L-1, k_scale_0..L-1]."""
    Ls = cell["layers"]
    return np.array([cell["amplitude"], cell["width"]] + [l["thickness"] for l in Ls]
                    + [l["k_scale"] for l in Ls], dtype=np.float64)


def with_params(cell, theta):
    """Copy of `cell` with theta (see params_of) applied."""
    import copy
    c = copy.deepcopy(cell)
    L = len(c["layers"])
    theta = np.asarray(theta, dtype=np.float64)
    c["amplitude"], c["width"] = float(theta[0]), float(theta[1])
    for m in range(L):
        c["layers"][m]["thickness"] = float(theta[2 + m])
        c["layers"][m]["k_scale"] = float(theta[2 + L + m])
    return c


_ADJOINT_SHAPES = {(2, 1), (4, 1), (8, 1), (4, 2), (8, 2), (4, 4), (8, 4)}


def _gradient_shape(cell):
    # one wave per line with 8 rows per lane up to nr = 512, else 4 rows per
    # lane over more waves (the adjoint kernels fit their registers there);
    # lines per wave as the plan picks them (about one workgroup per compute
    # unit), so that the adjoint's axial pass carries faces along each block
    nr, nz = int(cell["nr"]), int(cell["nz"])
    if nr <= 512:
        rpl, w = (2, 1) if nr <= 128 else ((4, 1) if nr <= 256 else (8, 1))
    else:
        rpl, w = 4, 1
        while 64 * 4 * w < nr:
            w *= 2
        if w > 4:
            return None
    lpw = min(8, max(1, int(round((nz - 2) / ((8 // w) * 256.0)))))
    return (rpl, w, lpw)


def gradient_plan(cell):
    """An FP64 plan of `cell` with the gradient's launch shape (set before
    the plan's first device use, as the library requires)."""
    plan = Plan(cell, "f64")
    sh = _gradient_shape(cell)
    if sh is not None:
        plan.set_shape(*sh)
    return plan


def gradient(cell, target, T0=None, nsteps=None, ckpt=0, store=0):
    """(J, dJ/dtheta, surface trace) of `cell` on the GPU (FP64); `store`
    kernel steps at the end keep their states (Plan.set_gradient_store)."""
    return gradient_plan(cell).gradient(target, T0=T0, nsteps=nsteps, ckpt=ckpt, store=store)


def gradient_many(cells, targets, nsteps=None, ckpt=0, streams=0, T0s=None, store=0, shared=0):
    """Gradients of many designs in one call (FP64, the library's concurrent
    design loop over `streams` HIP streams; 0 lets the library choose).
    Returns (J [n], [grad_i],
    [surface trace_i]); equal bit for bit to gradient() per design.  `store`:
    the gradient store of every design's plan (a number, or one per design).
    `shared` k > 0: k workspaces, design i on workspace i mod k (designs on
    one workspace run one after another), instead of one per design."""
    torch = _torch()
    n = len(cells)
    N = int(cells[0]["nsteps"] if nsteps is None else nsteps)
    plans, fields, sizes, tg = [], [], [], []
    for i, c in enumerate(cells):
        plan = gradient_plan(c)
        plan.set_gradient_store(store[i] if isinstance(store, (list, tuple)) else store)
        plans.append(plan)
        fields.append(plan.init() if T0s is None or T0s[i] is None else plan.field_from(T0s[i]))
        b = C.c_size_t()
        check(lib().cryo_gradient_workspace_bytes(plan._h, N, int(ckpt), C.byref(b)))
        sizes.append(b.value)
        t = np.ascontiguousarray(np.asarray(targets[i], dtype=np.float64)[:N])
        if t.size < N:
            raise ValueError("target %d needs nsteps values" % i)
        tg.append(t)
    k = int(shared)
    if k > 0:
        pool = [torch.empty(max(sizes[i::k]), dtype=torch.uint8, device="cuda")
                for i in range(min(k, n))]
        wss = [pool[i % k] for i in range(n)]
    else:
        wss = [torch.empty(sz, dtype=torch.uint8, device="cuda") for sz in sizes]
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    grads = [np.zeros(2 + 2 * len(c["layers"])) for c in cells]
    surfs = [np.zeros(N) for _ in cells]
    J = np.zeros(n)
    torch.cuda.synchronize()
    check(lib().cryo_gradient_many(
        n, (vp * n)(*[p._h for p in plans]), (vp * n)(*[_ptr(f) for f in fields]), N,
        (dp * n)(*[t.ctypes.data_as(dp) for t in tg]), int(ckpt),
        (vp * n)(*[_ptr(w) for w in wss]), (C.c_size_t * n)(*[w.numel() for w in wss]),
        int(streams), J.ctypes.data_as(dp), (dp * n)(*[g.ctypes.data_as(dp) for g in grads]),
        (dp * n)(*[x.ctypes.data_as(dp) for x in surfs])))
    return J, grads, surfs


def _make_solve():
    import torch

    class CryoSolve(torch.autograd.Function):
        """J(theta) for theta = [amplitude, width, thickness_m, k_scale_m] of a
        cell, differentiable by the hand-written discrete adjoint (one forward
        with checkpoints, recompute and adjoint sweep per call; `store` kernel
        steps at the end keep their states instead, see
        Plan.set_gradient_store).

        CryoSolve.apply(theta, cell, target, nsteps, ckpt[, store]) -> J (0-d
        tensor)."""

        @staticmethod
        def forward(ctx, theta, cell, target, nsteps, ckpt, store=0):
            c = with_params(cell, theta.detach().cpu().numpy())
            J, g, _ = gradient(c, target, nsteps=nsteps, ckpt=ckpt, store=store)
            ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
            return torch.as_tensor(J, dtype=theta.dtype, device=theta.device)

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            return gJ * g, None, None, None, None, None

    return CryoSolve


class _LazySolve:
    _cls = None

    def __getattr__(self, name):
        if _LazySolve._cls is None:
            _LazySolve._cls = _make_solve()
        return getattr(_LazySolve._cls, name)


CryoSolve = _LazySolve()
