"""ctypes binding of libdvm_hip.so (argument marshalling only).

Every function here maps one-to-one onto an ``extern "C"`` entry point of
include/dvm.h.  torch is imported first so that the HIP runtime torch loads is
the one the library binds to (both export the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime before the library)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdvm_hip.so")

DVM_OK, DVM_NOT_CONVERGED = 0, 1
DVM_ERR_ARG, DVM_ERR_STATE, DVM_ERR_OOM, DVM_ERR_DEVICE, DVM_ERR_NONPHYSICAL = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "DVM_OK", 1: "DVM_NOT_CONVERGED", -1: "DVM_ERR_ARG", -2: "DVM_ERR_STATE",
                -3: "DVM_ERR_OOM", -4: "DVM_ERR_DEVICE", -5: "DVM_ERR_NONPHYSICAL"}
DVM_F64, DVM_F32 = 0, 1


class DvmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class VGrid(C.Structure):
    _fields_ = [("m", C.c_int * 3), ("vmax", C.c_double * 3)]


class Gas(C.Structure):
    _fields_ = [("kn", C.c_double), ("omega", C.c_double), ("pr", C.c_double),
                ("conservative_correction", C.c_int)]


class FaceBC(C.Structure):
    _fields_ = [("kind", C.c_int), ("u", C.c_double * 3), ("T", C.c_double), ("rho", C.c_double)]


class Info(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("ncells", C.c_int),
                ("nfluid", C.c_int), ("m", C.c_int * 3), ("nvel", C.c_int), ("precision", C.c_int),
                ("brick", C.c_int * 3), ("vel_per_lane", C.c_int), ("tiles_per_octant", C.c_int),
                ("sweep_launches", C.c_int), ("workspace_bytes", C.c_size_t), ("pipelined", C.c_int),
                ("velocity_groups", C.c_int), ("parameter_bits", C.c_int), ("sweep_streams", C.c_int)]


_P = C.POINTER(C.c_double)
EXPORTS = {
    "dvm_create": ([C.POINTER(Grid), C.POINTER(VGrid), C.POINTER(Gas), C.c_int, C.c_void_p,
                    C.POINTER(C.c_void_p)], C.c_int),
    "dvm_set_face_bc": ([C.c_void_p, C.c_int, C.POINTER(FaceBC)], C.c_int),
    "dvm_set_solid": ([C.c_void_p, C.c_void_p, _P, C.c_double], C.c_int),
    "dvm_set_solid_mask": ([C.c_void_p, C.c_void_p, _P, C.c_double], C.c_int),
    "dvm_set_schedule": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "dvm_set_parameter_precision": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_set_sweep_streams": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_set_closed": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_set_spacing": ([C.c_void_p, _P, _P, _P], C.c_int),
    "dvm_set_velocity_groups": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_set_order": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_set_model": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_get_stress": ([C.c_void_p, _P], C.c_int),
    "dvm_set_stress": ([C.c_void_p, _P], C.c_int),
    "dvm_set_velocity_axes": ([C.c_void_p, _P, _P, _P, _P, _P, _P], C.c_int),
    "dvm_required_workspace": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "dvm_bind_workspace": ([C.c_void_p, C.c_void_p, C.c_size_t], C.c_int),
    "dvm_bind_static_workspace": ([C.c_void_p], C.c_int),
    "dvm_init_uniform": ([C.c_void_p, C.c_double, _P, C.c_double], C.c_int),
    "dvm_init_fields": ([C.c_void_p, _P, _P, _P, C.c_double], C.c_int),
    "dvm_iterate": ([C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_int), _P], C.c_int),
    "dvm_get_residuals": ([C.c_void_p, _P], C.c_int),
    "dvm_get_fields": ([C.c_void_p, _P, _P, _P, _P], C.c_int),
    "dvm_get_state": ([C.c_void_p, _P, _P, _P, _P], C.c_int),
    "dvm_set_state": ([C.c_void_p, _P, _P, _P, C.c_double], C.c_int),
    "dvm_get_info": ([C.c_void_p, C.POINTER(Info)], C.c_int),
    "dvm_set_timing": ([C.c_void_p, C.c_int], C.c_int),
    "dvm_get_timings": ([C.c_void_p, _P, _P, _P, C.POINTER(C.c_int)], C.c_int),
    "dvm_get_launch_timings": ([C.c_void_p, _P, C.POINTER(C.c_longlong)], C.c_int),
    "dvm_selftest_wave_reduce": ([_P, _P], C.c_int),
    "dvm_last_error": ([], C.c_char_p),
    "dvm_destroy": ([C.c_void_p], None),
}

_lib = None


def lib():
    """Load libdvm_hip.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1810_00348_amd.build.build() "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int):
    if status < 0:
        raise DvmError(status, lib().dvm_last_error().decode())
    return status
