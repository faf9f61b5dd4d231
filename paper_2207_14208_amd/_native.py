"""ctypes binding of libbcmg.so: the functions of include/bcmg.h under the same
names, argument marshalling only.  Every computation runs in the HIP library;
if it is not built this module raises ImportError (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bcmg.h")

OK, ERR_INVALID, ERR_OOM, ERR_DEVICE, ERR_NOT_CONVERGED, ERR_DIVERGED, ERR_STATE = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "OOM", 3: "DEVICE", 4: "NOT_CONVERGED", 5: "DIVERGED", 6: "STATE"}
OUTSIDE, INSIDE, GHOST, BOXDIR = 0, 1, 2, 3
FP64, MIXED = 0, 1
DTAU_OPT_EXP, DTAU_OPT_POLY, DTAU_CONST = 0, 1, 2
RESTRICT_RENORM_FW, RESTRICT_PLAIN_MEAN = 0, 1
BC_DIRICHLET, BC_NEUMANN = 0, 1
LAYOUT_NATURAL, LAYOUT_SPLIT = 0, 1
CYCLE_V, CYCLE_W = 0, 1
SMOOTH_RB, SMOOTH_JACOBI = 0, 1
PARAM_COARSE_NODES = 1
PARAM_LDS_BYTES = 2
PARAM_SWEEP_PAIR_SEGS = 3
LDS_DEFAULT = 150 * 1024


class bcmg_options(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("coarsest_N", C.c_int32), ("max_cycles", C.c_int32),
                ("precision", C.c_int32), ("dtau_mode", C.c_int32), ("dtau_const", C.c_double),
                ("ext_iters", C.c_int32), ("restrict_mode", C.c_int32), ("seg_len", C.c_int32),
                ("bc", C.c_int32), ("reaction", C.c_double), ("layout", C.c_int32), ("cycle", C.c_int32),
                ("smoother", C.c_int32), ("check_interval", C.c_int32)]


class bcmg_solve_stats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("status", C.c_int32), ("r0", C.c_double), ("r_final", C.c_double),
                ("rho_mean", C.c_double), ("solve_ms", C.c_double)]


class BcmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bcmg status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
P = C.POINTER

PROTOTYPES = {
    "bcmg_last_error": (C.c_char_p, []),
    "bcmg_version": (i32, []),
    "bcmg_default_options": (i32, [P(bcmg_options)]),
    "bcmg_setup": (i32, [i32, i32, vp, P(bcmg_options), vp, P(vp)]),
    "bcmg_destroy": (i32, [vp]),
    "bcmg_num_levels": (i32, [vp, P(i32)]),
    "bcmg_level_info": (i32, [vp, i32, P(i32), P(i64), P(i64), P(i64), P(i64)]),
    "bcmg_classes": (i32, [vp, i32, vp]),
    "bcmg_ghost_info": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
    "bcmg_ghost_stats": (i32, [vp, i32, P(i64), P(i64), P(i64)]),
    "bcmg_set_data": (i32, [vp, vp, vp]),
    "bcmg_fill_boundary": (i32, [vp, vp, vp]),
    "bcmg_vcycle": (i32, [vp, vp]),
    "bcmg_residual_norm": (i32, [vp, vp, P(dbl)]),
    "bcmg_residual_norm_noalloc": (i32, [vp, vp, P(dbl)]),
    "bcmg_solve": (i32, [vp, vp, dbl, P(bcmg_solve_stats), vp]),
    "bcmg_level_smooth": (i32, [vp, i32, vp, vp, i32]),
    "bcmg_level_residual": (i32, [vp, i32, vp, vp, vp, P(dbl)]),
    "bcmg_level_extend": (i32, [vp, i32, vp]),
    "bcmg_level_restrict": (i32, [vp, i32, vp, vp]),
    "bcmg_level_prolong": (i32, [vp, i32, vp, vp]),
    "bcmg_coarse_solve": (i32, [vp, vp, vp]),
    "bcmg_batch_create": (i32, [i32, vp, P(vp)]),
    "bcmg_batch_destroy": (i32, [vp]),
    "bcmg_batch_add": (i32, [vp, vp, vp, dbl, P(i32)]),
    "bcmg_batch_remove": (i32, [vp, i32]),
    "bcmg_batch_restart": (i32, [vp]),
    "bcmg_batch_step": (i32, [vp, i32, vp]),
    "bcmg_batch_run": (i32, [vp, i32, i32]),
    "bcmg_batch_stats": (i32, [vp, i32, P(bcmg_solve_stats), vp]),
    "bcmg_estimate_bytes": (i32, [i32, i32, i32, P(i64)]),
    "bcmg_batch_set_param": (i32, [vp, i32, i64]),
    "bcmg_problem_bytes": (i32, [vp, P(i64)]),
    "bcmg_timing_enable": (i32, [i32]),
    "bcmg_timing_read": (i32, [P(i64), P(dbl), P(i64)]),
    "bcmg_timing_sweeps": (i32, [vp, vp, i32, P(dbl)]),
    "bcmg_set_allocator": (i32, [vp, vp, vp]),
}

# callback types of bcmg_set_allocator: alloc(bytes, stream, ctx) -> ptr, free(ptr, bytes, stream, ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


def header_functions() -> list[str]:
    """Names of the functions declared in include/bcmg.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcmg_[a-z_0-9]+)\s*\(", text)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, allow=(OK,)) -> int:
    if status not in allow:
        raise BcmgError(status, lib().bcmg_last_error().decode())
    return status


def default_options(**kw) -> bcmg_options:
    o = bcmg_options()
    check(lib().bcmg_default_options(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o
