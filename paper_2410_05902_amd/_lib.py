"""ctypes binding of libmbkk.so (include/mbkk.h).  Argument marshalling only.

The library must have been built (paper_2410_05902_amd/csrc/build.py); there
is no fallback of any kind: loading fails loudly when the .so is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbkk.so")

OK, E_INVALID, E_STATE, E_WORKSPACE, E_HIP, E_INDEX, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
GAUSS, LAPLACE, LINEAR, POLY2 = 0, 1, 2, 3
FP32, FP64, BF16X3, BF16X1 = 0, 1, 2, 3
LR_BETA, LR_FULL, LR_SKLEARN = 0, 1, 2
CROSS_AUTO, CROSS_DIRECT, CROSS_MFMA = 0, 1, 2

EXPORTS = [
    "mbkk_workspace_size", "mbkk_create", "mbkk_destroy", "mbkk_last_error", "mbkk_set_data",
    "mbkk_init_centers", "mbkk_init_kmeanspp", "mbkk_step", "mbkk_assign", "mbkk_objective",
    "mbkk_get_state", "mbkk_set_state", "mbkk_center_norms", "mbkk_set_timing", "mbkk_get_timing",
    "mbkk_objective_fwd", "mbkk_objective_bwd", "mbkk_last_batch_objective", "mbkk_agreement",
    "mbkk_rescore_count", "mbkk_selfnorm_error_bound", "mbkk_create_static",
    "mbkk_microbench",  # include/mbkk_microbench.h
]
PROBE_SUBADD, PROBE_FMA, PROBE_EXP2, PROBE_MFMA_BF16, PROBE_MFMA_F32, PROBE_MFMA_BF16_CHAIN = 0, 1, 2, 3, 4, 5


class MbkkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mbkk error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("d", C.c_int32), ("k", C.c_int32), ("b_max", C.c_int32),
        ("window", C.c_int32), ("kernel", C.c_int32), ("kernel_param", C.c_double),
        ("precision", C.c_int32), ("lr", C.c_int32), ("cross_impl", C.c_int32),
        ("tie_delta", C.c_double), ("validate", C.c_int32), ("tau", C.c_int32),
    ]


class State(C.Structure):
    _fields_ = [
        ("iteration", C.c_int64), ("k", C.c_int32), ("window", C.c_int32), ("b_max", C.c_int32),
        ("init_idx", C.POINTER(C.c_int32)), ("slot_b", C.POINTER(C.c_int32)),
        ("slot_idx", C.POINTER(C.c_int32)), ("slot_off", C.POINTER(C.c_int32)),
        ("coef", C.POINTER(C.c_double)), ("cum", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    """Loads libmbkk.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2410_05902_amd.csrc.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.mbkk_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.mbkk_create.argtypes = [C.POINTER(Config), P, C.c_size_t, P, C.POINTER(P)]
        L.mbkk_destroy.argtypes = [P]
        L.mbkk_last_error.argtypes = [P]
        L.mbkk_last_error.restype = C.c_char_p
        L.mbkk_set_data.argtypes = [P, P, I64]
        L.mbkk_init_centers.argtypes = [P, P]
        L.mbkk_init_kmeanspp.argtypes = [P, P, P]
        L.mbkk_step.argtypes = [P, P, I32, P, P, C.POINTER(D)]
        L.mbkk_assign.argtypes = [P, P, I64, P, P, P, P]
        L.mbkk_objective.argtypes = [P, P, I64, C.POINTER(D)]
        L.mbkk_last_batch_objective.argtypes = [P, C.POINTER(D)]
        L.mbkk_agreement.argtypes = [P, P, P, I64, I32, P, C.POINTER(D), C.POINTER(D)]
        L.mbkk_get_state.argtypes = [P, C.POINTER(State)]
        L.mbkk_set_state.argtypes = [P, C.POINTER(State)]
        L.mbkk_center_norms.argtypes = [P, P]
        L.mbkk_set_timing.argtypes = [P, I32]
        L.mbkk_get_timing.argtypes = [P, C.POINTER(D), C.POINTER(I64)]
        L.mbkk_objective_fwd.argtypes = [P, P, I32, D, P, C.POINTER(D)]
        L.mbkk_objective_bwd.argtypes = [P, P, I32, D, P, D, P, C.POINTER(D)]
        L.mbkk_rescore_count.argtypes = [P, C.POINTER(I64), I32]
        L.mbkk_selfnorm_error_bound.argtypes = [P, C.POINTER(D)]
        L.mbkk_create_static.argtypes = [C.POINTER(Config), P, C.POINTER(P)]
        L.mbkk_microbench.argtypes = [I32, I64, I32, P, P, C.POINTER(D), C.POINTER(D)]
        for name in EXPORTS:
            if name != "mbkk_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int, ctx=None):
    if rc != OK:
        msg = lib().mbkk_last_error(ctx)
        raise MbkkError(rc, msg.decode() if msg else "")
