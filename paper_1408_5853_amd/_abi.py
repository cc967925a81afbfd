"""ctypes declarations of the cryocell C ABI (include/cryocell.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when libcryocell.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcryocell.so")

CRYO_OK = 0
STATUS = {0: "CRYO_OK", 1: "CRYO_ERR_ARG", 2: "CRYO_ERR_UNSTABLE", 3: "CRYO_ERR_DEVICE",
          4: "CRYO_ERR_NONFINITE", 5: "CRYO_ERR_WORKSPACE", 6: "CRYO_ERR_UNSUPPORTED"}
F64, F32 = 0, 1

# every exported symbol the header declares
SYMBOLS = [
    "cryo_last_error", "cryo_version", "cryo_validate", "cryo_stability_dt_max",
    "cryo_plan_create", "cryo_plan_destroy", "cryo_grid_radii", "cryo_source_fraction",
    "cryo_workspace_bytes", "cryo_init", "cryo_forward", "cryo_poll",
    "cryo_plan_shape", "cryo_plan_set_shape", "cryo_plan_set_turn_on", "cryo_plan_set_poly_laws",
    "cryo_plan_set_stepped", "cryo_plan_set_gradient_store", "cryo_gradient_store_steps",
    "cryo_batch_create", "cryo_batch_create_with", "cryo_batch_destroy", "cryo_batch_offsets", "cryo_batch_shape",
    "cryo_batch_workspace_bytes", "cryo_batch_init", "cryo_batch_forward", "cryo_batch_poll",
    "cryo_gradient_workspace_bytes", "cryo_gradient", "cryo_gradient_async", "cryo_gradient_many",
    "cryo_autotune", "cryo_batch_autotune", "cryo_batch_autotune_with",
    "cryo_state_create", "cryo_state_destroy", "cryo_state_load", "cryo_state_forward",
    "cryo_state_store", "cryo_forward_noalloc",
]


class CryoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Material(C.Structure):
    _fields_ = [("k0", C.c_double), ("p", C.c_double), ("k_scale", C.c_double),
                ("c0", C.c_double), ("q", C.c_double), ("rho", C.c_double),
                ("tref", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("thickness", C.c_double), ("intervals", C.c_int32), ("mat", Material)]


class Geometry(C.Structure):
    _fields_ = [("r_inner", C.c_double), ("height", C.c_double), ("nr", C.c_int32),
                ("nz", C.c_int32), ("n_layers", C.c_int32), ("layers", C.POINTER(Layer))]


class Pulse(C.Structure):
    _fields_ = [("layer", C.c_int32), ("amplitude", C.c_double), ("width", C.c_double),
                ("period", C.c_double), ("t_on", C.c_double)]


class Boundary(C.Structure):
    _fields_ = [("kind", C.c_int32 * 4), ("value", C.c_double * 4)]


class Problem(C.Structure):
    _fields_ = [("geom", Geometry), ("pulse", Pulse), ("bc", Boundary), ("dt", C.c_double),
                ("T_init", C.c_double)]


class InstanceOptions(C.Structure):
    _fields_ = [("poly_a", C.POINTER(C.c_double)), ("poly_b", C.POINTER(C.c_double)),
                ("joule_tref", C.c_double), ("z_full", C.c_int32), ("nr_top", C.c_int32),
                ("turn_on", C.c_int32)]


_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcryocell.so is not built; run paper_1408_5853_amd/build.py "
                              "(or __graft_entry__.build())")
        # torch ships its own HIP runtime (same soname as the system one);
        # load it first so that the process holds exactly one runtime and
        # the tensors torch allocates live on the device this library sees
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
        pp = C.POINTER(Problem)
        L.cryo_last_error.restype = C.c_char_p
        L.cryo_version.restype = C.c_char_p
        L.cryo_validate.argtypes = [pp]
        L.cryo_stability_dt_max.argtypes = [pp, C.c_double, dp]
        L.cryo_plan_create.argtypes = [pp, C.c_int, C.POINTER(vp)]
        L.cryo_plan_destroy.argtypes = [vp]
        L.cryo_plan_destroy.restype = None
        L.cryo_grid_radii.argtypes = [vp, dp]
        L.cryo_source_fraction.argtypes = [vp, i64, i64, dp]
        L.cryo_workspace_bytes.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
        L.cryo_init.argtypes = [vp, vp, vp]
        L.cryo_forward.argtypes = [vp, vp, i64, i64, vp, C.c_size_t, vp, vp]
        L.cryo_poll.argtypes = [vp, vp, vp]
        L.cryo_forward_noalloc.argtypes = [vp, vp, i64, i64, vp, vp]
        L.cryo_state_create.argtypes = [vp, vp, C.c_size_t, C.POINTER(vp)]
        L.cryo_state_destroy.argtypes = [vp]
        L.cryo_state_destroy.restype = None
        L.cryo_state_load.argtypes = [vp, vp, vp]
        L.cryo_state_forward.argtypes = [vp, i64, i64, vp, vp]
        L.cryo_state_store.argtypes = [vp, vp, vp]
        i32p = C.POINTER(C.c_int32)
        L.cryo_plan_shape.argtypes = [vp, i32p, i32p, i32p]
        L.cryo_plan_set_shape.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.cryo_plan_set_turn_on.argtypes = [vp, C.c_int32]
        L.cryo_plan_set_poly_laws.argtypes = [vp, dp, dp, C.c_double]
        L.cryo_plan_set_stepped.argtypes = [vp, C.c_int32, C.c_int32]
        L.cryo_plan_set_gradient_store.argtypes = [vp, i64]
        L.cryo_gradient_store_steps.argtypes = [vp, i64, i64, C.c_size_t, C.POINTER(C.c_int64)]
        L.cryo_batch_create.argtypes = [C.c_int32, pp, C.c_int, i32p, C.POINTER(vp)]
        L.cryo_batch_create_with.argtypes = [C.c_int32, pp, C.c_int, i32p,
                                             C.POINTER(InstanceOptions), C.POINTER(vp)]
        L.cryo_batch_destroy.argtypes = [vp]
        L.cryo_batch_destroy.restype = None
        L.cryo_batch_offsets.argtypes = [vp, C.POINTER(C.c_int64)]
        L.cryo_batch_shape.argtypes = [vp, C.c_int32, i32p]
        L.cryo_batch_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.cryo_batch_init.argtypes = [vp, vp, vp]
        L.cryo_batch_forward.argtypes = [vp, vp, i64, i64, vp, C.c_size_t, vp]
        L.cryo_batch_poll.argtypes = [vp, vp, vp, i32p]
        L.cryo_autotune.argtypes = [pp, C.c_int, C.c_int32, C.c_char_p, vp, i32p, dp]
        L.cryo_batch_autotune.argtypes = [C.c_int32, pp, C.c_int, C.c_int32, C.c_char_p, vp,
                                          i32p]
        L.cryo_batch_autotune_with.argtypes = [C.c_int32, pp, C.c_int,
                                               C.POINTER(InstanceOptions), C.c_int32,
                                               C.c_char_p, vp, i32p]
        L.cryo_gradient_workspace_bytes.argtypes = [vp, i64, i64, C.POINTER(C.c_size_t)]
        L.cryo_gradient.argtypes = [vp, vp, i64, dp, i64, vp, C.c_size_t, dp, dp, dp, vp]
        L.cryo_gradient_async.argtypes = [vp, vp, i64, vp, i64, vp, C.c_size_t, vp, vp, vp, vp]
        L.cryo_gradient_many.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), i64,
                                         C.POINTER(dp), i64, C.POINTER(vp),
                                         C.POINTER(C.c_size_t), C.c_int32, dp, C.POINTER(dp),
                                         C.POINTER(dp)]
        for name in SYMBOLS:
            if name not in ("cryo_last_error", "cryo_version", "cryo_plan_destroy",
                            "cryo_batch_destroy", "cryo_state_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status):
    if status != CRYO_OK:
        raise CryoError(status, lib().cryo_last_error().decode())


class ProblemStruct:
    """A Problem structure built from a problem dictionary; keeps its layer
    array alive."""

    def __init__(self, cell):
        Ls = cell["layers"]
        self.layers = (Layer * len(Ls))()
        for m, l in enumerate(Ls):
            self.layers[m].thickness = float(l["thickness"])
            self.layers[m].intervals = int(l["intervals"])
            mt = self.layers[m].mat
            mt.k0, mt.p, mt.k_scale = float(l["k0"]), float(l["p"]), float(l["k_scale"])
            mt.c0, mt.q = float(l["c0"]), float(l["q"])
            mt.rho, mt.tref = float(l["rho"]), float(l["tref"])
        s = Problem()
        s.geom.r_inner = float(cell["r_inner"])
        s.geom.height = float(cell["height"])
        s.geom.nr, s.geom.nz = int(cell["nr"]), int(cell["nz"])
        s.geom.n_layers = len(Ls)
        s.geom.layers = C.cast(self.layers, C.POINTER(Layer))
        s.pulse.layer = int(cell["heater"])
        s.pulse.amplitude = float(cell["amplitude"])
        s.pulse.width = float(cell["width"])
        s.pulse.period = float(cell["period"])
        s.pulse.t_on = float(cell["t_on"])
        for q in range(4):
            s.bc.kind[q] = int(cell["bc"][q][0])
            s.bc.value[q] = float(cell["bc"][q][1])
        s.dt = float(cell["dt"])
        s.T_init = float(cell["T_init"])
        self.s = s

    def ref(self):
        return C.byref(self.s)
