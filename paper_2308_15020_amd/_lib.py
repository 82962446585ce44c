"""ctypes binding of libffsat.so (argument marshalling only).

The library must have been built in-tree (``paper_2308_15020_amd/lib``);
there is no fallback: every call runs the HIP kernels or raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "lib", "libffsat.so")
HEADER = os.path.join(ROOT, "include", "ffsat.h")

STATUS = {
    0: "OK", -1: "E_INVALID_ARG", -2: "E_VAR_RANGE", -3: "E_DUP_VAR", -4: "E_EMPTY_CONSTRAINT",
    -5: "E_BAD_KIND", -6: "E_DEVICE_MISMATCH", -7: "E_NOMEM", -8: "E_HIP", -9: "E_NONFINITE",
    -10: "E_UNSUPPORTED",
}

FLAG_FORCE_DFT = 1
FLAG_DEBUG_CHECKS = 4
FLAG_UNIT_CIRCLE = 8
MAX_CONSTRAINT_LEN = 512


class FFSatError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.code = STATUS.get(status, str(status))


class ProblemDesc(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_cons", C.c_int32), ("con_ptr", C.c_void_p),
                ("lits", C.c_void_p), ("kinds", C.c_void_p), ("params", C.c_void_p),
                ("weights", C.c_void_p), ("device", C.c_int32), ("fp64_min_len", C.c_int32),
                ("flags", C.c_uint32)]


class ProblemInfo(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_cons", C.c_int32), ("nnz", C.c_int64),
                ("max_len", C.c_int32), ("n_bins_f32", C.c_int32), ("n_bins_f64", C.c_int32),
                ("device", C.c_int32), ("device_bytes", C.c_int64)]


class MpnnDesc(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("rounds", C.c_int32), ("device", C.c_int32),
                ("reserved", C.c_int32), ("seed", C.c_uint64)]


class PlanOpts(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("use_graphs", C.c_int32), ("tune_cache", C.c_char_p),
                ("reserved", C.c_int32 * 8)]


_lib = None

P = C.c_void_p
I32 = C.c_int32

_SIGS = {
    "ffsat_status_string": (C.c_char_p, [I32]),
    "ffsat_last_error": (C.c_char_p, []),
    "ffsat_version": (C.c_char_p, []),
    "ffsat_problem_create": (I32, [C.POINTER(ProblemDesc), C.POINTER(P)]),
    "ffsat_problem_destroy": (I32, [P]),
    "ffsat_problem_info_get": (I32, [P, C.POINTER(ProblemInfo)]),
    "ffsat_set_weights": (I32, [P, P, I32, P]),
    "ffsat_get_weights": (I32, [P, P, I32, P]),
    "ffsat_plan_create": (I32, [P, I32, C.POINTER(PlanOpts), C.POINTER(P)]),
    "ffsat_plan_destroy": (I32, [P]),
    "ffsat_plan_tune": (I32, [P, P]),
    "ffsat_plan_describe": (I32, [P, C.c_char_p, C.c_size_t]),
    "ffsat_eval": (I32, [P, P, P, P, P, P]),
    "ffsat_eval_f64": (I32, [P, P, P, P, P, P]),
    "ffsat_eval_check": (I32, [P, P, P, P, P, P, P, P, P]),
    "ffsat_eval_noalloc": (I32, [P, I32, P, P, P, P]),
    "ffsat_eval_step": (I32, [P, P, C.c_float, P, P, P, P]),
    "ffsat_step": (I32, [P, P, P, P, C.c_float, P]),
    "ffsat_step_f64": (I32, [P, P, P, P, C.c_double, P]),
    "ffsat_run_steps": (I32, [P, P, I32, C.c_float, P, P]),
    "ffsat_round_check": (I32, [P, P, P, P, P, P, P]),
    "ffsat_round_check_f64": (I32, [P, P, P, P, P, P, P]),
    "ffsat_erwa_update": (I32, [P, P, C.c_float, P]),
    "ffsat_weight_grad": (I32, [P, P, P, P, P]),
    "ffsat_coefficients": (I32, [I32, I32, I32, P]),
    "ffsat_walsh_coefficients": (I32, [I32, I32, I32, P]),
    "ffsat_unit_circle_coefficients": (I32, [I32, I32, I32, P]),
    "ffsat_vjp": (I32, [P, P, P, P, P, P, P]),
    "ffsat_rephase": (I32, [P, P, I32, C.c_uint64, P, P]),
    "ffsat_plan_profile": (I32, [P, I32]),
    "ffsat_plan_profile_read": (I32, [P, I32, C.c_char_p, C.c_size_t]),
    "ffsat_fista": (I32, [P, P, P, P, P, I32, I32, P, P]),
    "ffsat_sat_weight": (I32, [P, P, P, P, P]),
    "ffsat_run_iters": (I32, [P, P, I32, C.c_float, C.c_float, P, P, P, P]),
    "ffsat_mpnn_create": (I32, [P, P]),
    "ffsat_mpnn_destroy": (I32, [P]),
    "ffsat_mpnn_num_params": (I32, [P, P]),
    "ffsat_mpnn_params": (I32, [P, P, I32, I32, I32, P]),
    "ffsat_mpnn_forward": (I32, [P, P, P, P]),
    "ffsat_mpnn_backward": (I32, [P, P, P, P, P]),
    "ffsat_mpnn_adam": (I32, [P, C.c_float, C.c_float, C.c_float, C.c_float, P]),
    "ffsat_mpnn_propose": (I32, [P, P, P, C.c_float, C.c_float, C.c_uint64, P]),
}


def header_symbols() -> list:
    """Function names declared in include/ffsat.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ffsat_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"HIP library not built: {LIB_PATH} is missing "
                "(run __graft_entry__.build() or python paper_2308_15020_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().ffsat_last_error().decode(errors="replace")
        raise FFSatError(status, msg)
