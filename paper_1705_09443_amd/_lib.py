"""ctypes binding of liblsweep.so (declarations in include/lsweep.h).

Argument marshalling only: every computation runs in the HIP library. The
library is loaded from this package directory; if it is missing it is built
once (hipcc cross-compiles for gfx950), and if that fails the import fails
loudly. There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsweep.so")

LS_OK, LS_E_INVALID, LS_E_NOMEM, LS_E_DEVICE, LS_E_SINGULAR, LS_E_NOCONV, LS_E_NUMERIC, LS_E_STATE = range(8)
STATUS_NAMES = ["LS_OK", "LS_E_INVALID", "LS_E_NOMEM", "LS_E_DEVICE", "LS_E_SINGULAR", "LS_E_NOCONV",
                "LS_E_NUMERIC", "LS_E_STATE"]
LS_FP64, LS_MIXED = 0, 1
LS_RHS_SOURCE, LS_RHS_INCIDENT = 0, 1
LS_SWEEP_INTERFACE, LS_SWEEP_SEQUENTIAL = 0, 1

c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
P_int = ctypes.POINTER(ctypes.c_int)
P_double = ctypes.POINTER(ctypes.c_double)


class LsGrid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int)]


class LsOptions(ctypes.Structure):
    _fields_ = [("precision", c_int), ("restart", c_int), ("max_iters", c_int), ("pml_C", c_double),
                ("freq_samples", c_int), ("autotune", c_int), ("hip_stream", c_void_p),
                ("sweep_schedule", c_int), ("fronts", c_int), ("block_size", c_int)]


class LsRhsInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("rel_residual", c_double), ("converged", c_int)]


class LsSetupInfo(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int), ("pml_width", c_int), ("layer_thickness", c_int),
                ("L", c_int), ("nslices", c_int), ("freq_samples", c_int), ("precision", c_int),
                ("omega", c_double), ("h", c_double), ("pml_C", c_double), ("freq_lo", c_double),
                ("freq_delta", c_double), ("fronts", c_int)]


class LsKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int), ("total_ms", c_double),
                ("columns", ctypes.c_longlong)]


class LsTuneLayer(ctypes.Structure):
    _fields_ = [("layer_thickness", c_int), ("nslices", c_int), ("iterations", c_int), ("setup_ms", c_double),
                ("solve_ms", c_double)]


class LsTuneKernels(ctypes.Structure):
    _fields_ = [("nrhs", c_int), ("slice_kernel", c_int), ("iface_kernel", c_int), ("apply_ms", c_double)]


class LsError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}: {message}")


_SIGNATURES = {
    "ls_default_options": (None, [ctypes.POINTER(LsOptions)]),
    "ls_setup": (c_int, [ctypes.POINTER(LsGrid), c_double, c_void_p, c_int, c_int, ctypes.POINTER(LsOptions),
                         ctypes.POINTER(c_void_p)]),
    "ls_solve": (c_int, [c_void_p, c_void_p, c_int, c_int, c_double, c_void_p, ctypes.POINTER(LsRhsInfo)]),
    "ls_adjoint": (c_int, [c_void_p, c_void_p, c_int, c_double, c_void_p, ctypes.POINTER(LsRhsInfo)]),
    "ls_destroy": (None, [c_void_p]),
    "ls_last_error": (ctypes.c_char_p, []),
    "ls_apply_A": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_apply_A_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_apply_B": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_solve_H": (c_int, [c_void_p, c_void_p, c_int, c_double, c_void_p, ctypes.POINTER(LsRhsInfo)]),
    "ls_apply_K": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_apply_Q": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_apply_H": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_apply_precond": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_slice_solve": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p, c_int]),
    "ls_get_info": (c_int, [c_void_p, ctypes.POINTER(LsSetupInfo)]),
    "ls_get_slice": (c_int, [c_void_p, c_int, P_int, P_int, P_int]),
    "ls_get_stencils": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ls_get_sample_map": (c_int, [c_void_p, c_void_p]),
    "ls_profile": (c_int, [c_void_p, c_int]),
    "ls_profile_read": (c_int, [c_void_p, ctypes.POINTER(LsKernelTime), c_int, P_int]),
    "ls_layer_candidates": (c_int, [c_int, c_int, P_int, c_int, P_int]),
    "ls_get_tuning": (c_int, [c_void_p, ctypes.POINTER(LsTuneLayer), c_int, P_int, ctypes.POINTER(LsTuneKernels),
                              c_int, P_int]),
    "ls_set_kernels": (c_int, [c_void_p, c_int, c_int, c_int]),
    "ls_host_tables": (c_int, [c_int, c_double, c_void_p, c_int, c_int, c_double, c_int, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p]),
    "ls_stencil_cache": (c_int, [c_int, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
    "ls_host_tables3": (c_int, [c_int, c_double, c_void_p, c_int, c_int, c_double, c_int, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p]),
    "ls_op3_create": (c_int, [c_int, c_double, c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "ls_op3_apply_A": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_op3_apply_K": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "ls_op3_destroy": (None, [c_void_p]),
    "ls_host_green3": (c_int, [c_int, c_double, c_void_p]),
}

_lib = None
_lock = threading.Lock()


def load(build_if_missing: bool = True) -> ctypes.CDLL:
    """Load liblsweep.so (building it first if it is absent)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            if not build_if_missing:
                raise RuntimeError(f"{LIB_PATH} is missing; run __graft_entry__.build()")
            from .build import build
            build()
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(status: int, where: str) -> int:
    if status not in (LS_OK,):
        raise LsError(status, where, load().ls_last_error().decode(errors="replace"))
    return status
