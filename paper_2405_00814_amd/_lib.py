"""ctypes binding of libgemfdtd.so: the C ABI declared in include/gemfdtd.h,
function for function and with the same names.  Argument marshalling only;
every step of the computation runs in the HIP library.  There is no
fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libgemfdtd.so")

FDTD_OK, FDTD_EINVAL, FDTD_EUNSTABLE, FDTD_ENOMEM, FDTD_EDEVICE, FDTD_ENONFINITE, FDTD_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
FDTD_EX, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ = range(6)
FDTD_SRC_GAUSSIAN, FDTD_SRC_RICKER, FDTD_SRC_TABLE = 0, 1, 2

STATUS_NAMES = {0: "FDTD_OK", -1: "FDTD_EINVAL", -2: "FDTD_EUNSTABLE", -3: "FDTD_ENOMEM",
                -4: "FDTD_EDEVICE", -5: "FDTD_ENONFINITE", -6: "FDTD_ESTATE"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class fdtd_allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class fdtd_cpml(C.Structure):
    _fields_ = [("npml", C.c_int32 * 6), ("m", C.c_double), ("sigma_max", C.c_double),
                ("kappa_max", C.c_double), ("alpha_max", C.c_double), ("m_alpha", C.c_double),
                ("split", C.c_int32)]


class fdtd_desc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("eps_r", C.POINTER(C.c_float)), ("mu_r", C.POINTER(C.c_float)),
                ("sigma", C.POINTER(C.c_float)), ("cpml", fdtd_cpml), ("stream", C.c_void_p),
                ("allocator", C.POINTER(fdtd_allocator))]


class fdtd_kernel_config(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tile", C.c_int32 * 4), ("tb", C.c_int32)]


class fdtd_launch_stat(C.Structure):
    _fields_ = [("ms", C.c_float), ("cells", C.c_int64), ("psi", C.c_int64), ("cpml", C.c_int32),
                ("launches", C.c_int32), ("steps", C.c_int32)]


class FdtdError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__("%s failed: %s (%s)" % (where, msg, STATUS_NAMES.get(code, code)))
        self.code = code


_lock = threading.Lock()
_L = None

P = C.c_void_p
i32, i64, f32p, f64p, i32p, i64p = C.c_int32, C.c_int64, C.POINTER(C.c_float), \
    C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)

_SIGS = {
    "fdtd_create": (C.c_int, [C.POINTER(fdtd_desc), C.POINTER(P)]),
    "fdtd_create_graph": (C.c_int, [C.POINTER(fdtd_desc), C.POINTER(P)]),
    "fdtd_destroy": (C.c_int, [P]),
    "fdtd_set_source": (C.c_int, [P, C.c_int, i32p, C.c_int, f64p, f32p, i64]),
    "fdtd_set_source_box": (C.c_int, [P, C.c_int, i32p, i32p, C.c_int, f64p, f32p, i64]),
    "fdtd_set_dft": (C.c_int, [P, C.c_int, i32p, i32p, C.c_int, f64p]),
    "fdtd_get_dft": (C.c_int, [P, f64p, f64p, C.POINTER(C.c_int64)]),
    "fdtd_dft_sar": (C.c_int, [P, f32p, f64p, f32p]),
    "fdtd_set_probes": (C.c_int, [P, C.c_int, i32p, i32]),
    "fdtd_step": (C.c_int, [P, i64]),
    "fdtd_probe": (C.c_int, [P, f32p, i64, i64p]),
    "fdtd_probe_noalloc": (C.c_int, [P, f32p, i64, i64p]),
    "fdtd_get_field": (C.c_int, [P, C.c_int, P, C.c_int]),
    "fdtd_set_field": (C.c_int, [P, C.c_int, P, C.c_int]),
    "fdtd_state_bytes": (C.c_int, [P, i64p]),
    "fdtd_save_state": (C.c_int, [P, P, C.c_int]),
    "fdtd_load_state": (C.c_int, [P, P, C.c_int]),
    "fdtd_reset": (C.c_int, [P]),
    "fdtd_steps_done": (C.c_int, [P, i64p]),
    "fdtd_check_finite": (C.c_int, [P]),
    "fdtd_set_material": (C.c_int, [P, i32p, i32p, f32p, f32p]),
    "fdtd_set_kernel": (C.c_int, [P, C.POINTER(fdtd_kernel_config)]),
    "fdtd_get_kernel": (C.c_int, [P, C.POINTER(fdtd_kernel_config)]),
    "fdtd_autotune": (C.c_int, [P, i32, C.POINTER(fdtd_kernel_config)]),
    "fdtd_last_step_time": (C.c_int, [P, C.POINTER(C.c_float), i64p]),
    "fdtd_step_profile": (C.c_int, [P, i32, C.POINTER(fdtd_launch_stat), i32, i32p]),
    "fdtd_batch_create": (C.c_int, [C.POINTER(fdtd_desc), i32, C.POINTER(P)]),
    "fdtd_batch_destroy": (C.c_int, [P]),
    "fdtd_batch_set_source": (C.c_int, [P, i32, i32p, C.c_int, f64p, f32p, i64]),
    "fdtd_batch_set_probes": (C.c_int, [P, i32, i32p, i32]),
    "fdtd_batch_step": (C.c_int, [P, i64]),
    "fdtd_batch_set_kernel": (C.c_int, [P, i32, i32, i32, i32]),
    "fdtd_batch_autotune": (C.c_int, [P, i32, i32p]),
    "fdtd_batch_probe": (C.c_int, [P, i32, f32p, i64, i64p]),
    "fdtd_batch_get_field": (C.c_int, [P, i32, C.c_int, P, C.c_int]),
    "fdtd_batch_last_step_time": (C.c_int, [P, C.POINTER(C.c_float), i64p]),
    "fdtd_batch_cells": (C.c_int, [P, i64p]),
    "fdtd_adjoint_eps": (C.c_int, [P, i64, i64, i64, i32p, i32, f64p, f32p]),
    "fdtd_adjoint": (C.c_int, [P, i64, i64, i64, i32p, i32, f64p, f32p, f32p]),
    "fdtd_adjoint_grads": (C.c_int, [P, i64, i64, i64, i32p, i32, f64p, f32p, f32p, f32p]),
    "fdtd_stream_copy": (C.c_int, [P, P, C.c_size_t, P]),
    "fdtd_last_error": (C.c_char_p, []),
    "fdtd_version": (C.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def open_library(path: str):
    """dlopen the HIP library at path and declare the signatures."""
    if not os.path.exists(path):
        raise RuntimeError("libgemfdtd.so not found at %s; build it with "
                           "`python -m paper_2405_00814_amd.build`" % path)
    L = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def load():
    """The process-wide library handle (raises if it has not been built).

    torch is imported first when it is installed: the library and torch then
    share torch's HIP runtime, whichever of the two the caller touches first
    (with the library loaded first, torch's device initialisation afterwards
    left the library's HIP calls without a device)."""
    global _L
    with _lock:
        if _L is None:
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            _L = open_library(LIBPATH)
    return _L


def check(code: int, where: str):
    if code != FDTD_OK:
        msg = load().fdtd_last_error().decode(errors="replace")
        raise FdtdError(code, where, msg)
    return code


def call(name: str, *args):
    """Call a C-ABI function by name and raise FdtdError on a nonzero status."""
    return check(getattr(load(), name)(*args), name)
