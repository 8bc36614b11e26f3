"""ctypes declarations of the C interface in ``include/polyeval.h``."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolyeval.so")

PE_FP64, PE_DD = 0, 1
PE_NEWTON_MIXED, PE_NEWTON_DD = 0, 1
STATUS = {0: "PE_OK", 1: "PE_EINVAL", 2: "PE_ENOMEM", 3: "PE_EDEVICE", 4: "PE_EUNSUPPORTED",
          5: "PE_ENOTCONVERGED"}


class PolyevalError(RuntimeError):
    def __init__(self, status, where, message):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {message}")


class pe_cvec(C.Structure):
    _fields_ = [("re_hi", C.c_void_p), ("re_lo", C.c_void_p), ("im_hi", C.c_void_p),
                ("im_lo", C.c_void_p)]


class pe_track_params(C.Structure):
    _fields_ = [("gamma_re", C.c_double), ("gamma_im", C.c_double), ("h_init", C.c_double),
                ("h_min", C.c_double), ("h_max", C.c_double), ("corr_tol", C.c_double),
                ("corr_iters", C.c_int32), ("max_steps", C.c_int32), ("end_tol", C.c_double),
                ("end_iters", C.c_int32)]


def cvec(ptrs):
    return pe_cvec(*[C.c_void_p(int(p)) if p else None for p in ptrs])


_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "pe_version": (C.c_char_p, []),
    "pe_last_error": (C.c_char_p, []),
    "pe_create_system": (C.c_int, [C.c_int32, C.c_int32, C.c_int64, _I64P, _I64P, _I32P, _I32P,
                                   pe_cvec, C.POINTER(C.c_void_p)]),
    "pe_destroy_system": (C.c_int, [C.c_void_p]),
    "pe_system_info": (C.c_int, [C.c_void_p, _I32P, _I32P, _I64P, _I32P, _I32P]),
    "pe_eval_jac": (C.c_int, [C.c_void_p, C.c_int64, pe_cvec, pe_cvec, pe_cvec, C.c_int,
                              C.c_void_p]),
    "pe_eval_jac_noalloc": (C.c_int, [C.c_void_p, C.c_int64, pe_cvec, pe_cvec, pe_cvec, C.c_int,
                                      C.c_void_p]),
    "pe_eval_jac_qd": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_void_p), C.c_void_p]),
    "pe_eval_jac_paper_layout": (C.c_int, [C.c_void_p, C.c_int64, pe_cvec, pe_cvec, pe_cvec, C.c_int,
                                           C.c_void_p]),
    "pe_set_schedule": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32]),
    "pe_get_schedule": (C.c_int, [C.c_void_p, C.c_int64, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "pe_newton": (C.c_int, [C.c_void_p, C.c_int64, pe_cvec, C.c_double, C.c_int32, C.c_int,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pe_newton_qd": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p), C.c_double,
                               C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pe_start_solutions": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, pe_cvec, C.c_void_p]),
    "pe_track": (C.c_int, [C.c_void_p, C.c_int64, pe_cvec, C.POINTER(pe_track_params), C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pe_create_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "pe_destroy_batch": (C.c_int, [C.c_void_p]),
    "pe_batch_layout": (C.c_int, [C.c_void_p, _I64P, _I64P, _I64P, _I64P]),
    "pe_eval_jac_batch": (C.c_int, [C.c_void_p, _I64P, pe_cvec, pe_cvec, pe_cvec, C.c_int,
                                    C.c_void_p]),
    "pe_batch_config": (C.c_int, [C.c_void_p, _I32P, _I32P, _I32P, _I32P]),
    "pe_autotune_batch": (C.c_int, [C.c_void_p, _I64P, pe_cvec, pe_cvec, pe_cvec, C.c_int,
                                    C.c_void_p, C.c_char_p]),
    "pe_autotune_system": (C.c_int, [C.c_void_p, C.c_int64, pe_cvec, pe_cvec, pe_cvec, C.c_int,
                                     C.c_void_p, C.c_char_p]),
}

_LIB = None


def lib():
    """Load libpolyeval.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1201_0499_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status, where):
    if status != 0:
        msg = lib().pe_last_error()
        raise PolyevalError(status, where, msg.decode() if msg else "")
