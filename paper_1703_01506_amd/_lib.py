"""ctypes loader for librpt.so: symbol table and status handling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpt.so")

_p = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u64 = C.c_uint64
_f32 = C.c_float
_sz = C.c_size_t
_int = C.c_int



class RptStudy(C.Structure):
    """Mirror of struct rpt_study (include/rpt.h), natural alignment."""
    _fields_ = [
        ("X", _p), ("v", _i64), ("n", _i32), ("n1", _i32), ("ldx", _i64), ("labels", _p), ("L_rec", _i64),
        ("col0", _i64), ("U", _p), ("r", _i32), ("study", C.c_uint32), ("sigma_mu", _p), ("omega_ptr", _p),
        ("omega_idx", _p), ("nnz", _i64), ("seed", _u64), ("max_out", _p), ("info", _p),
    ]


class RptTracker(C.Structure):
    """Mirror of rpt_tracker (include/rpt.h)."""
    _fields_ = [("kind", _i32), ("rho", C.c_float), ("admm_iters", _i32)]


# name -> (restype, argtypes); mirrors include/rpt.h
SIGNATURES = {
    "rpt_status_string": (C.c_char_p, [_int]),
    "rpt_last_hip_error": (_int, []),
    "rpt_version": (_int, []),
    "rpt_timing_enable": (None, [_int]),
    "rpt_timing_reset": (None, []),
    "rpt_timing_query": (_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "rpt_timing_stages": (_int, [C.c_char_p, _sz]),
    "rpt_naive_workspace": (_sz, [_i64, _i32, _i64, _int]),
    "rpt_naive_maxnull": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i64, _int, _int, _int, _p, _p, _p, _sz, _p]),
    "rpt_sampled_tstat_workspace": (_sz, [_i64, _i32]),
    "rpt_sampled_tstat": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i64, _p, _i32, _int, _p, _p, _sz, _p]),
    "rpt_complete_workspace": (_sz, [_i64, _i32]),
    "rpt_complete": (_int, [_p, _i64, _i32, _p, _i32, _p, _i64, _p, _p, _p, _p, _sz, _p]),
    "rpt_train_workspace": (_sz, [_i64, _i32, _i32, _i32, _i32, _int]),
    "rpt_train_subspace": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i32, _p, _i32, _p, _i32, _i32, _i32, _f32,
                                  C.c_double, _p, _u64, _int, _int, _int, C.POINTER(RptTracker), _p, _p, _p, _p,
                                  _p, _p, _p, _p, _sz, _p]),
    "rpt_sigma_mu_workspace": (_sz, [_i64, _i32, _i32, _i32, _i32, _int]),
    "rpt_sigma_mu": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i32, _p, _i32, _p, _i32, _u64, _int, _int, _int, _p,
                            _p, _p, _p, _sz, _p]),
    "rpt_recover_workspace": (_sz, [_i64, _i32, _i64, _i32, _i32]),
    "rpt_autotune_naive": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i64, _int, _p, _i32, _p, _sz, _p, _p]),
    "rpt_autotune_recover_workspace": (_sz, [_i64, _i32, _i64]),
    "rpt_autotune_recover": (_int, [_i64, _i32, _i64, _i32, _p, _sz, _p, _p]),
    "rpt_autotune_save": (_int, [C.c_char_p]),
    "rpt_autotune_load": (_int, [C.c_char_p]),
    "rpt_autotune_clear": (None, []),
    "rpt_autotune_count": (_int, []),
    "rpt_rapidpt_workspace": (_sz, [_i64, _i32, _i32, _i64, _i32, _i32, _int]),
    "rpt_rapidpt_gen_workspace": (_sz, [_i32, _i32, _i64, _i32, _i32]),
    "rpt_sample_count": (_i64, [_i64, _i32]),
    "rpt_gen_relabellings": (_int, [_u64, _i64, _i64, _i32, _i32, _p, _p]),
    "rpt_gen_sampled_sets": (_int, [_u64, _i32, _i64, _i64, _i64, _i32, _p, _p]),
    "rpt_gen_start_basis": (_int, [_u64, _i64, _i32, _p, _p]),
    "rpt_rapidpt_maxnull": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i32, _p, _i64, _p, _i32, _p, _i32, _i32, _i32,
                                   _f32, C.c_double, _p, _p, _u64, _int, _int, _int, C.POINTER(RptTracker), _p, _p,
                                   _p, _p, _p, _p, _p, _p, _sz, _p]),
    "rpt_recover_maxnull": (_int, [_p, _i64, _i32, _i64, _i32, _p, _i64, _i64, _p, _i32, _p, _p, _i32, _p, _u64,
                                   _int, _p, _p, _p, _p, _sz, _p]),
    "rpt_recover_batched_workspace": (_sz, [C.POINTER(RptStudy), _i32]),
    "rpt_recover_maxnull_batched": (_int, [C.POINTER(RptStudy), _i32, _p, _sz, _p]),
    "rpt_observed_tstat_workspace": (_sz, [_i64, _i32]),
    "rpt_observed_tstat": (_int, [_p, _i64, _i32, _i64, _i32, _p, _p, _sz, _p]),
    "rpt_fwer_threshold": (_int, [_p, _i64, C.c_double, _p, _p]),
    "rpt_corrected_pvalues": (_int, [_p, _i64, _p, _i64, _p, _p]),
    "rpt_rejection_counts": (_int, [_p, _i64, _p, _i64, _p, _i64, C.c_double, _p, _p]),
    "rpt_reorth_workspace": (_sz, [_i64, _i32]),
    "rpt_reorth": (_int, [_p, _i64, _i32, _p, _p, _sz, _p]),
    "rpt_reorth_noalloc_capacity": (_sz, []),
    "rpt_reorth_noalloc": (_int, [_p, _i64, _i32, _p, _p]),
    "rpt_masked_loss_fwd": (_int, [_p, _i64, _i32, _p, _i32, _p, _p, _p, _i64, _p, _p, _p]),
    "rpt_masked_loss_bwd": (_int, [_p, _i64, _i32, _p, _i32, _p, _p, _p, _i64, _p, _p, _p, _p]),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load librpt.so (once).  Raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"librpt.so not found at {path}; build it with `python paper_1703_01506_amd/build.py`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RPTError(RuntimeError):
    def __init__(self, code: int, what: str):
        lib = load()
        msg = lib.rpt_status_string(code).decode()
        if code == -5:
            msg += f" (hipError {lib.rpt_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]")
        self.code = code


def check(code: int, what: str) -> None:
    if code != 0:
        raise RPTError(code, what)
