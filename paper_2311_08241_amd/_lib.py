"""ctypes view of include/sesub.h (argument marshalling only).

Loads the in-tree libsesub.so; raises ImportError when it has not been built,
so no code path can silently fall back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsesub.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sesub.h")

c_int64, c_int32, c_uint32, c_double, c_void_p = (ctypes.c_int64, ctypes.c_int32,
                                                   ctypes.c_uint32, ctypes.c_double,
                                                   ctypes.c_void_p)

SE_OK, SE_ERR_ARG, SE_ERR_MESH, SE_ERR_HIP, SE_ERR_OOM, SE_ERR_CFL = 0, 1, 2, 3, 4, 5
SE_ERR_DRY, SE_ERR_NONFINITE, SE_ERR_UNSUPPORTED = 6, 7, 8
SE_F64, SE_F32_MIXED = 0, 1
SE_SCHEME_SE, SE_SCHEME_SESM = 0, 1
SE_PERIODIC_X, SE_PERIODIC_Y, SE_SPHERICAL = 1, 2, 4
SE_LINEAR_H, SE_CHECK_CFL, SE_TRACK_VOLUME = 1, 2, 4
SE_FAULT_DRY, SE_FAULT_NONFINITE, SE_FAULT_LAYERS = 1, 2, 4

STATUS_NAMES = {0: "SE_OK", 1: "SE_ERR_ARG", 2: "SE_ERR_MESH", 3: "SE_ERR_HIP", 4: "SE_ERR_OOM",
                5: "SE_ERR_CFL", 6: "SE_ERR_DRY", 7: "SE_ERR_NONFINITE", 8: "SE_ERR_UNSUPPORTED"}


class MeshDesc(ctypes.Structure):
    _fields_ = [("nv", c_int64), ("ne", c_int64), ("x", c_void_p), ("y", c_void_p),
                ("tri", c_void_p), ("flags", c_uint32), ("period_x", c_double),
                ("period_y", c_double), ("radius", c_double)]


class Params(ctypes.Structure):
    _fields_ = [("g", c_double), ("theta", c_double), ("precision", c_int32),
                ("flags", c_uint32), ("eta_ref", c_double), ("h_max", c_double),
                ("scheme", c_int32), ("reserved", c_int32), ("beta", c_double),
                ("delta", c_double), ("gamma", c_double), ("zeta", c_double),
                ("visc_A0", c_double), ("visc_Cv", c_double)]


class State(ctypes.Structure):
    _fields_ = [("eta", c_void_p), ("U", c_void_p), ("Uavg", c_void_p), ("volume", c_void_p)]


class Forcing(ctypes.Structure):
    _fields_ = [("R", c_void_p), ("f", c_void_p), ("H0", c_void_p), ("W", c_void_p)]


class PlanStats(ctypes.Structure):
    _fields_ = [("ntiles", c_int32), ("max_tri", c_int32), ("max_vtx", c_int32),
                ("tri_per_thread", c_int32), ("lds_f32", c_int32), ("lds_f64", c_int32),
                ("ok_f32", c_int32), ("ok_f64", c_int32), ("tri_overhead", c_double),
                ("vtx_overhead", c_double), ("bytes_per_vs_f32", c_double),
                ("bytes_per_vs_f64", c_double), ("lds_sesm_f32", c_int32),
                ("lds_sesm_f64", c_int32), ("ok_sesm_f32", c_int32), ("ok_sesm_f64", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

_SIGS = {
    "se_last_error": (ctypes.c_char_p, []),
    "se_sesm_coefficients": (c_int32, [c_double, c_double, c_void_p]),
    "se_mesh_create": (c_int32, [ctypes.POINTER(MeshDesc), c_int32, ctypes.POINTER(c_void_p)]),
    "se_mesh_destroy": (None, [c_void_p]),
    "se_mesh_info": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "se_mesh_perm": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "se_mesh_csr": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "se_mesh_neighbours": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "se_mesh_geometry": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "se_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(Params), c_int32, c_int32,
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "se_subcycle": (c_int32, [c_void_p, ctypes.POINTER(Params), ctypes.POINTER(State),
                              ctypes.POINTER(Forcing), c_int32, c_double, c_void_p, c_void_p]),
    "se_subcycle_noalloc": (c_int32, [c_void_p, ctypes.POINTER(Params), ctypes.POINTER(State),
                                      ctypes.POINTER(Forcing), c_int32, c_double, c_void_p]),
    "se_subcycle_plain": (c_int32, [c_void_p, ctypes.POINTER(Params), ctypes.POINTER(State),
                                    ctypes.POINTER(Forcing), c_int32, c_double, c_void_p,
                                    c_void_p]),
    "se_subcycle_adjoint": (c_int32, [c_void_p, ctypes.POINTER(Params), c_void_p, c_void_p,
                                      ctypes.POINTER(Forcing), c_int32, c_double, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p]),
    "se_trim_zstar": (c_int32, [c_void_p, c_int32] + [c_void_p] * 7 + [c_double] +
                      [c_void_p] * 4),
    "se_barotropic_visc": (c_int32, [c_void_p, c_int32, ctypes.c_uint32, c_double, c_double,
                                     c_double] + [c_void_p] * 6),
    "se_forcing_assemble": (c_int32, [c_void_p, c_int32] + [c_void_p] * 6 + [c_double, c_int32] +
                   [c_void_p] * 2),
    "se_batch_create": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p)]),
    "se_batch_destroy": (None, [c_void_p]),
    "se_batch_info": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "se_batch_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(Params), c_void_p,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "se_subcycle_batched": (c_int32, [c_void_p, ctypes.POINTER(Params), ctypes.POINTER(State),
                                      ctypes.POINTER(Forcing), c_void_p, c_void_p, c_int32,
                                      c_void_p, c_void_p]),
    "se_set_plan": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32]),
    "se_get_plan": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "se_check_faults": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "se_plan_stats": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32,
                                ctypes.POINTER(PlanStats)]),
}


def header_functions():
    """Names of the functions declared in include/sesub.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(se_[a-z_]+)\s*\(", src)))


def lib():
    """The loaded library; ImportError if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != SE_OK:
        raise SeError(status, lib().se_last_error().decode(errors="replace"))
