"""ctypes declarations of the libcgd C-ABI (include/cgd.h)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcgd.so")

MAX_FIELDS = 16
MAX_STEPS = 64

OK = 0
NOT_CONVERGED = 1
WARMSTART_FALLBACK = 2
E_INVALID = -1
E_NONFINITE = -2
E_NOMEM = -3
E_HIP = -4
E_BREAKDOWN = -5
E_UNSUPPORTED = -6

c_mesh = ctypes.c_void_p
c_unet = ctypes.c_void_p


class SolverOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("x0_mode", ctypes.c_int32), ("x0", ctypes.c_void_p),
                ("check_every", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("scheme", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("n_fields", ctypes.c_int32),
                ("iters", (ctypes.c_int32 * MAX_FIELDS) * MAX_STEPS),
                ("rel_res", (ctypes.c_double * MAX_FIELDS) * MAX_STEPS),
                ("mass_before", ctypes.c_double * MAX_FIELDS),
                ("mass_after", ctypes.c_double * MAX_FIELDS),
                ("frac_bits", ctypes.c_int32 * MAX_FIELDS),
                ("n_dropped", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64),
                ("status", ctypes.c_int32), ("n_fallback", ctypes.c_int32)]


TIMING_KINDS = 18


class KernelTiming(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * TIMING_KINDS),
                ("total_ms", ctypes.c_double * TIMING_KINDS),
                ("bytes_per_launch", ctypes.c_double * TIMING_KINDS)]


# name -> (restype, argtypes)
SIGNATURES = {
    "cgd_mesh_create_hex": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(c_mesh)]),
    "cgd_mesh_create_tet": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.POINTER(c_mesh)]),
    "cgd_mesh_create_tet_d": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(c_mesh)]),
    "cgd_mesh_create_rect": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.POINTER(c_mesh)]),
    "cgd_mesh_destroy": (None, [c_mesh]),
    "cgd_mesh_num_cells": (ctypes.c_int64, [c_mesh]),
    "cgd_mesh_kind": (ctypes.c_int32, [c_mesh]),
    "cgd_mesh_nnz": (ctypes.c_int64, [c_mesh]),
    "cgd_locate": (ctypes.c_int32, [c_mesh, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "cgd_deposit": (ctypes.c_int32, [c_mesh, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.POINTER(SolveStats), ctypes.c_void_p]),
    "cgd_deposit_noalloc": (ctypes.c_int32, [c_mesh, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cgd_diffuse": (ctypes.c_int32, [c_mesh, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_int32, ctypes.POINTER(SolverOpts),
                                     ctypes.POINTER(SolveStats), ctypes.c_void_p]),
    "cgd_coarse_grain": (ctypes.c_int32, [c_mesh, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                          ctypes.POINTER(SolverOpts), ctypes.c_void_p,
                                          ctypes.POINTER(SolveStats), ctypes.c_void_p]),
    "cgd_coarse_grain_batched": (ctypes.c_int32, [c_mesh, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                                  ctypes.c_int32, ctypes.POINTER(SolverOpts), ctypes.c_void_p,
                                                  ctypes.POINTER(SolveStats), ctypes.c_void_p]),
    "cgd_velocity_from_momentum": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "cgd_autotune_batched": (ctypes.c_int32, [c_mesh, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "cgd_unet_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.POINTER(c_unet)]),
    "cgd_unet_destroy": (None, [c_unet]),
    "cgd_unet_num_params": (ctypes.c_int64, [c_unet]),
    "cgd_unet_get_params": (ctypes.c_int32, [c_unet, ctypes.c_void_p, ctypes.c_int64]),
    "cgd_unet_set_params": (ctypes.c_int32, [c_unet, ctypes.c_void_p, ctypes.c_int64]),
    "cgd_unet_get_grads": (ctypes.c_int32, [c_unet, ctypes.c_void_p, ctypes.c_int64]),
    "cgd_unet_forward": (ctypes.c_int32, [c_unet, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cgd_unet_loss_grad": (ctypes.c_int32, [c_unet, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "cgd_unet_train_step": (ctypes.c_int32, [c_unet, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "cgd_conv3_forward": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cgd_conv3_dgrad": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "cgd_conv3_wgrad": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "cgd_timing_enable": (ctypes.c_int32, [c_mesh, ctypes.c_int32]),
    "cgd_timing_read": (ctypes.c_int32, [c_mesh, ctypes.POINTER(KernelTiming), ctypes.c_int32]),
    "cgd_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "cgd_last_error": (ctypes.c_char_p, []),
    "cgd_version": (ctypes.c_int32, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libcgd.so (raises if it has not been built) and declares its symbols."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcgd.so not found at {path}: build it with "
                          "`python -m paper_1409_0001_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
