"""ctypes binding of libdirac.so: argument marshalling only.

Every function here has the name of the C entry point it calls (see
include/dirac.h for argument meaning, layout, ownership and errors).  A missing
library raises ImportError; nothing falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdirac.so")

DIRAC_C64 = 1
DIRAC_C128 = 2
DIRAC_ALLOW_UNSTABLE = 1
DIRAC_SLAB_Z = 2
DIRAC_ZERO_BC = 4
DIRAC_KERNEL_AUTO, DIRAC_KERNEL_SPLIT, DIRAC_KERNEL_FUSED, DIRAC_KERNEL_FUSED2 = 0, 1, 2, 3
DIRAC_E_STATE = -6
STATUS = {0: "DIRAC_OK", -1: "DIRAC_E_ARG", -2: "DIRAC_E_SHAPE", -3: "DIRAC_E_UNSTABLE",
          -4: "DIRAC_E_NONFINITE", -5: "DIRAC_E_HIP", -6: "DIRAC_E_STATE"}

#: every entry point of include/dirac.h
EXPORTS = (
    "dirac_status_string", "dirac_create", "dirac_destroy", "dirac_last_error", "dirac_bind_state",
    "dirac_current", "dirac_set_current", "dirac_halo_steps", "dirac_scratch_bytes", "dirac_bind_scratch",
    "dirac_set_mass_potential_z", "dirac_theta_from_fields", "dirac_set_theta_field", "dirac_set_kernel",
    "dirac_step", "dirac_step_norm", "dirac_reverse", "dirac_norm_device", "dirac_norm", "dirac_observables",
    "dirac_seed_region", "dirac_adjoint_vz", "dirac_batch_create", "dirac_batch_bind", "dirac_batch_run",
    "dirac_batch_norms", "dirac_batch_autotune", "dirac_coef_from_theta", "dirac_set_potential_im_z",
    "dirac_coef_from_theta_c", "dirac_set_links", "dirac_coef_from_fields", "dirac_set_mass",
    "dirac_set_potential_z", "dirac_adjoint", "dirac_autotune", "dirac_coef_from_theta_host",
    "dirac_norm_device_static", "dirac_batch_create_dt", "dirac_stream_copy",
)


class DiracError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, message))


_lib = None


def lib():
    """The loaded library (ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdirac.so is not built (run paper_1309_3452_amd/build.py): " + LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I64, D, I, U = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_uint
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "dirac_status_string": ([I], ctypes.c_char_p),
        "dirac_create": ([ctypes.POINTER(P), I, I64, I64, I64, I, D, D, D, D, U], I),
        "dirac_destroy": ([P], None),
        "dirac_last_error": ([P], ctypes.c_char_p),
        "dirac_bind_state": ([P, PP, PP], I),
        "dirac_current": ([P, ctypes.POINTER(I)], I),
        "dirac_set_current": ([P, I], I),
        "dirac_halo_steps": ([P, ctypes.POINTER(I)], I),
        "dirac_scratch_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], I),
        "dirac_bind_scratch": ([P, P, ctypes.c_size_t], I),
        "dirac_set_mass_potential_z": ([P, D, P, P, I64], I),
        "dirac_theta_from_fields": ([P, D, PP, PP, P], I),
        "dirac_set_theta_field": ([P, PP], I),
        "dirac_set_kernel": ([P, I, I, I], I),
        "dirac_step": ([P, I64, P], I),
        "dirac_reverse": ([P, I64, P], I),
        "dirac_step_norm": ([P, I64, P, P], I),
        "dirac_norm_device": ([P, P, P], I),
        "dirac_norm_device_static": ([P, P, P], I),
        "dirac_norm": ([P, ctypes.POINTER(D), P], I),
        "dirac_observables": ([P, D, ctypes.POINTER(D), P], I),
        "dirac_seed_region": ([P, D, PP, P], I),
        "dirac_adjoint_vz": ([P, I64, PP, P, P, P], I),
        "dirac_adjoint": ([P, I64, PP, D, P, P, P], I),
        "dirac_set_mass": ([P, D], I),
        "dirac_set_potential_z": ([P, P, P, I64], I),
        "dirac_autotune": ([P, ctypes.c_char_p], I),
        "dirac_batch_create": ([ctypes.POINTER(P), I64, ctypes.POINTER(I64), ctypes.POINTER(I64), I, D, U], I),
        "dirac_batch_create_dt": ([ctypes.POINTER(P), I64, ctypes.POINTER(I64), ctypes.POINTER(I64), I,
                                   ctypes.POINTER(D), U], I),
        "dirac_batch_bind": ([P, PP, PP, PP, P, ctypes.c_size_t], I),
        "dirac_batch_run": ([P, I64, I, I, P], I),
        "dirac_batch_norms": ([P, ctypes.POINTER(D), P], I),
        "dirac_batch_autotune": ([P, ctypes.c_char_p, ctypes.POINTER(I), P], I),
        "dirac_coef_from_theta": ([P, P, I64, P], I),
        "dirac_stream_copy": ([P, P, I64, P], I),
        "dirac_coef_from_theta_host": ([P, P, I64], I),
        "dirac_coef_from_theta_c": ([P, P, P, I64, P], I),
        "dirac_set_potential_im_z": ([P, P, P, I64], I),
        "dirac_set_links": ([P, PP], I),
        "dirac_coef_from_fields": ([P, I, D, D, P, P, I64, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * max(1, len(ptrs)))()
    for q, p in enumerate(ptrs):
        arr[q] = p
    return arr


def check(rc, ctx=None):
    if rc != 0:
        msg = ""
        if ctx is not None:
            m = lib().dirac_last_error(ctx)
            msg = m.decode() if m else ""
        raise DiracError(rc, msg)
    return rc
