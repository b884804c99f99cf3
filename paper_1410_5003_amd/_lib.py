"""ctypes binding of include/mlh.h (argument marshalling only).

Every computation happens in libmlh.so on the GPU.  If the library has not
been built, loading raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlh.so")
ABI_VERSION = 2

MLH_IFACE_FOURIER = 0
MLH_IFACE_POLYGON = 1

STATUS = {0: "MLH_OK", 1: "MLH_E_INVALID_ARG", 2: "MLH_E_GEOMETRY", 3: "MLH_E_NOMEM",
          4: "MLH_E_DEVICE", 5: "MLH_E_SINGULAR", 6: "MLH_E_ACCURACY", 7: "MLH_E_UNSUPPORTED"}

PIECES = {"A_self": 0, "A_up": 1, "A_dn": 2, "B_own": 3, "B_below": 4, "C_own": 5, "C_above": 6,
          "Q": 7, "Z_U": 8, "Z_D": 9, "V_U": 10, "V_D": 11}


class MlhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, str(status)), msg))
        self.status = status


class mlh_interface(C.Structure):
    _fields_ = [("kind", C.c_int32), ("y0", C.c_double), ("n_modes", C.c_int32),
                ("cos_coef", C.POINTER(C.c_double)), ("sin_coef", C.POINTER(C.c_double)),
                ("n_nodes", C.c_int32), ("n_vert", C.c_int32),
                ("vx", C.POINTER(C.c_double)), ("vy", C.POINTER(C.c_double)),
                ("seg_nodes", C.POINTER(C.c_int32)), ("q", C.c_double)]


class mlh_stack_desc(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("I", C.c_int32), ("iface", C.POINTER(mlh_interface)),
                ("k", C.POINTER(C.c_double)), ("d", C.c_double), ("y_U", C.c_double),
                ("y_D", C.c_double), ("P", C.c_int32), ("R", C.c_double), ("M_w", C.c_int32),
                ("M_ud", C.c_int32), ("K", C.c_int32), ("ls_mu", C.c_double)]


class mlh_profile(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "fill_self_ms", "fill_alpert_ms", "fill_pairs_ms", "assemble_ms", "rb_setup_ms", "ls_panel_ms",
        "ls_update_ms", "ls_rhs_ms", "schur_ms", "sweep_gemm_ms", "gje_panel_ms", "gje_update_ms", "gje_rhs_ms", "backsub_ms",
        "bragg_ms")] + \
        [("n_sweep_gemm", C.c_int32), ("n_gje_panel", C.c_int32), ("n_gje_update", C.c_int32),
         ("total_ms", C.c_double), ("gje_step_ms", C.c_double), ("n_gje_step", C.c_int32),
         ("n_schur_gemm", C.c_int32), ("n_gje_rhs", C.c_int32), ("n_backsub", C.c_int32),
         ("schur_flops", C.c_double), ("sweep_gemm_flops", C.c_double), ("gje_step_flops", C.c_double),
         ("gje_panel_update_flops", C.c_double), ("gje_rhs_flops", C.c_double)]


class mlh_tuning(C.Structure):
    _fields_ = [("rhs_in_step_pct", C.c_int32), ("ls_row_blocks", C.c_int32), ("gje_rhs_cols", C.c_int32),
                ("asm_in_panels", C.c_int32), ("gemm_slab_k", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "mlh_ctx_create": (C.c_int32, [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mlh_ctx_destroy": (C.c_int32, [C.c_void_p]),
    "mlh_stack_create": (C.c_int32, [C.c_void_p, C.POINTER(mlh_stack_desc), C.POINTER(C.c_void_p)]),
    "mlh_stack_refill": (C.c_int32, [C.c_void_p]),
    "mlh_stack_destroy": (C.c_int32, [C.c_void_p]),
    "mlh_stack_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]),
    "mlh_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mlh_solve_noalloc": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mlh_stack_set_flux_tolerance": (C.c_int32, [C.c_void_p, C.c_double]),
    "mlh_field": (C.c_int32, [C.c_void_p, C.c_double, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.c_int32, C.c_void_p, C.c_void_p]),
    "mlh_adjoint": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.c_void_p]),
    "mlh_batch_create": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "mlh_batch_destroy": (C.c_int32, [C.c_void_p]),
    "mlh_batch_solve": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mlh_batch_get_tuning": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mlh_batch_set_tuning": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mlh_batch_autotune": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_void_p]),
    "mlh_batch_tune_cached": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "mlh_debug_get_piece": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32)]),
    "mlh_debug_hankel": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "mlh_debug_zgemm": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mlh_debug_solve_partial": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32]),
    "mlh_debug_get_work": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "mlh_profile_step": (C.c_int32, [C.c_void_p, C.c_double, C.c_void_p]),
    "mlh_profile_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p]),
    "mlh_stack_get_tuning": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mlh_stack_set_tuning": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mlh_stack_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.c_void_p]),
    "mlh_stack_tune_cached": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p,
                                          C.POINTER(C.c_int32)]),
    "mlh_last_error": (C.c_char_p, []),
}


def lib():
    """Load libmlh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmlh.so not found at %s: run paper_1410_5003_amd/build.py "
                              "(or __graft_entry__.build()) first" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != 0:
        raise MlhError(status, lib().mlh_last_error().decode())


def dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))
