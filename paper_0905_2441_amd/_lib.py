"""ctypes loader for libsmcgpu.so (built in-tree by ``paper_0905_2441_amd.build``).

There is no fallback: if the shared library is missing or fails to load, this
module raises, and so does everything that imports it.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_int, c_int32, c_int64, c_uint32,
                    c_uint64, c_void_p)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsmcgpu.so")

SMC_KMAX = 8
SMC_DMAX = 8
SMC_KDMAX = 64

SMC_OK = 0
SMC_ERR_INVALID_ARG = -1
SMC_ERR_UNSUPPORTED = -2
SMC_ERR_HIP = -3
SMC_ERR_NUMERIC = -4
SMC_ERR_NOMEM = -5
SMC_ERR_CAPTURE = -6

SMC_PREC_FP64 = 0
SMC_PREC_FP32 = 1
SMC_PREC_BF16X3 = 2

SMC_RESAMPLE_SYSTEMATIC = 0
SMC_RESAMPLE_STRATIFIED = 1
SMC_RESAMPLE_MULTINOMIAL = 2

SMC_PRIOR_GAUSS = 0
SMC_PRIOR_BOX = 1

SMC_RULE_CALL = 0
SMC_RULE_BATCH = 1


class SmcGmm(Structure):
    _fields_ = [("k", c_int32), ("d", c_int32), ("sigma2", c_double),
                ("log_w", c_double * SMC_KMAX), ("prior", c_int32),
                ("prior_a", c_double), ("prior_b", c_double)]


class SmcRunDesc(Structure):
    _fields_ = [("p_off", c_int64), ("y_off", c_int64), ("N", c_int32), ("n", c_int32),
                ("seed", c_uint64)]


SMC_FSV_MMAX = 8
SMC_FSV_KMAX = 4


class SmcFsv(Structure):
    _fields_ = [("m", c_int32), ("k", c_int32), ("B", c_double * (SMC_FSV_MMAX * SMC_FSV_KMAX)),
                ("psi", c_double * SMC_FSV_MMAX), ("phi", c_double * SMC_FSV_KMAX),
                ("U", c_double * (SMC_FSV_KMAX * SMC_FSV_KMAX))]


class SmcLaunchRule(Structure):
    _fields_ = [("k", c_int32), ("d", c_int32), ("prec", c_int32), ("kind", c_int32),
                ("slices", c_int32), ("n_lo", c_int64), ("n_hi", c_int64), ("N_lo", c_int64),
                ("N_hi", c_int64)]


_P = c_void_p
_GP = POINTER(SmcGmm)

# name -> (restype, argtypes); every function declared in include/smc.h and
# include/smc_fsv.h.
SIGNATURES = {
    "smc_create": (c_int, [POINTER(c_void_p), c_int]),
    "smc_destroy": (c_int, [_P]),
    "smc_reserve": (c_int, [_P, c_int64, c_int32, c_int64]),
    "smc_check": (c_int, [_P, _P]),
    "smc_last_error": (c_char_p, []),
    "smc_set_slices": (c_int, [_P, c_int32]),
    "pt_set_single_workgroup": (c_int, [_P, c_int32]),
    "smc_set_launch_table": (c_int, [_P, POINTER(SmcLaunchRule), c_int32]),
    "smc_fp32_form_counts": (c_int, [_P, POINTER(c_uint64), c_int32]),
    "smc_loglik": (c_int, [_P, _GP, _P, c_int64, _P, c_int64, c_int, _P, _P]),
    "smc_prior_init": (c_int, [_P, _GP, c_int64, c_uint64, _P, _P]),
    "smc_rwmh_move": (c_int, [_P, _GP, _P, c_int64, _P, _P, c_int64, _P, c_double, c_double,
                              c_uint64, c_uint64, c_uint32, c_int, _P, _P]),
    "smc_reweight": (c_int, [_P, _P, _P, c_int64, c_double, _P, _P, _P, _P]),
    "smc_ess": (c_int, [_P, _P, c_int64, _P, _P]),
    "smc_resample_systematic": (c_int, [_P, _P, c_int64, c_uint64, c_uint64, _P, _P, c_double,
                                        _P, _P, _P, c_int32, _P, _P, _P, _P]),
    "smc_resample": (c_int, [_P, c_int, _P, c_int64, c_uint64, c_uint64, _P, c_double, _P, _P,
                             _P, c_int32, _P, _P, _P, _P]),
    "smc_set_resampling": (c_int, [_P, c_int]),
    "smc_resample_noalloc": (c_int, [c_int, _P, c_int64, c_uint64, c_uint64, _P, c_double, _P,
                                     _P, _P, c_int32, _P, _P, _P, _P]),
    "pt_exchange": (c_int, [_P, _P, _P, _P, c_int64, c_int32, c_int32, c_int32, c_uint64,
                            c_uint64, _P, _P]),
    "pt_iterations": (c_int, [_P, _GP, _P, c_int64, c_int64, _P, _P, _P, _P, c_int32, c_double,
                              c_uint64, c_int32, c_int32, c_int, _P, _P, _P]),
    "pt_record": (c_int, [_P, _P, c_int64, c_int32, c_int64, _P, _P, c_int64, _P]),
    "fsv_init": (c_int, [_P, c_int32, c_int64, _P, _P, _P]),
    "fsv_step": (c_int, [_P, POINTER(SmcFsv), _P, c_int32, c_int64, _P, _P, _P, _P, c_uint64,
                         c_double, _P, _P, _P]),
    "fsv_steps": (c_int, [_P, POINTER(SmcFsv), _P, c_int32, c_int64, _P, _P, _P, _P, c_int32,
                          c_uint64, c_double, _P, _P, _P]),
    "smc_step": (c_int, [_P, _GP, _P, c_int64, c_int64, _P, _P, _P, _P, _P, _P, _P, c_int32, _P,
                         c_double, c_int32, c_uint64, c_double, c_int, _P, _P, _P]),
    "smc_steps": (c_int, [_P, _GP, _P, c_int64, c_int64, _P, _P, _P, _P, _P, _P, _P, c_int32, _P,
                          c_int32, c_double, c_int32, c_uint64, c_double, c_int, _P, _P, _P]),
    "pt_iteration": (c_int, [_P, _GP, _P, c_int64, c_int64, _P, _P, _P, _P, c_double, c_uint64,
                             c_int32, c_int32, c_int, _P, _P, _P]),
    "smc_batch_create": (c_int, [_P, POINTER(SmcRunDesc), c_int32, c_int32, POINTER(c_void_p)]),
    "smc_batch_destroy": (c_int, [_P]),
    "smc_step_batched": (c_int, [_P, _P, _GP, _P, _P, _P, _P, _P, _P, c_int32, _P, c_double,
                                 c_int32, c_double, c_int, _P, _P, _P]),
    "smc_graph_begin": (c_int, [_P, _P]),
    "smc_graph_end": (c_int, [_P, _P, POINTER(c_void_p)]),
    "smc_graph_launch": (c_int, [_P, _P]),
    "smc_graph_destroy": (c_int, [_P]),
    "smc_sort_data": (c_int, [_P, c_int64, _P]),
    "smc_rng_words": (c_int, [c_uint64, c_int64, c_uint32, c_uint32, c_uint32, c_uint32, _P, _P]),
    "smc_rng_normals": (c_int, [c_uint64, c_int64, c_int32, c_uint32, c_uint32, c_uint32, _P,
                                _P]),
}


class SmcError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"libsmcgpu error {code}: {message}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libsmcgpu.so once; raise ImportError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_0905_2441_amd/build.py` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != SMC_OK:
        msg = load().smc_last_error()
        raise SmcError(code, msg.decode() if msg else "")
