"""ctypes loader and signatures of ``libpolarbp.so``."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpolarbp.so")

PC_OK, PC_EINVAL, PC_ENOTSUP, PC_EHIP, PC_ENOMEM = 0, -1, -2, -3, -4
STOP_NONE, STOP_G, STOP_CRC = 0, 1, 2
PP_NONE, PP_LASTK, PP_FULL, PP_ALG1 = -1, 0, 1, 2
PP_ALG1_ORIG = 3  # Algorithm 1 with subgraphs of the original graph

# symbols declared in include/polarbp.h
EXPORTS = [
    "polar_construct", "polar_code_free", "polar_code_query", "polar_trellis_pool",
    "polar_encode", "bp_decode", "pp_mt_bp_decode", "pp_mt_bp_decode_ex",
    "polar_batched_workspace_bytes", "pp_mt_bp_decode_batched", "wbp_workspace_bytes",
    "wbp_forward", "wbp_backward", "polar_strerror", "polar_last_error",
    "pp_mt_bp_decode_trace", "polar_classify_errors", "polar_info_bits",
    "pp_mt_bp_decode_batched_noalloc",
]
CHECK_MINSUM, CHECK_EXACT = 0, 1
ERR_CORRECT, ERR_FALSE_CONVERGED, ERR_OSCILLATION, ERR_UNCONVERGED = 0, 1, 2, 3


class PolarError(RuntimeError):
    def __init__(self, rc: int, where: str):
        self.rc = rc
        detail = ""
        try:
            detail = lib().polar_last_error().decode()
            name = lib().polar_strerror(rc).decode()
        except Exception:  # library unusable: report the code only
            name = str(rc)
        super().__init__(f"{where}: {name} ({rc}): {detail}")


class BPParamsC(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("stop", ctypes.c_int32), ("it_min", ctypes.c_int32), ("check", ctypes.c_int32)]


class PPParamsC(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("k", ctypes.c_int32), ("period_T", ctypes.c_int32),
                ("pool_Q", ctypes.c_int32), ("P_range", ctypes.c_int32),
                ("P_level", ctypes.c_int32), ("D", ctypes.c_int32), ("N_min", ctypes.c_int32),
                ("first_reset", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("noise_sigma", ctypes.c_float)]


class LaunchCfgC(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_int32), ("slots", ctypes.c_int32), ("grid", ctypes.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_1911_08868_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u32, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t)
    P = ctypes.POINTER
    sig = {
        "polar_construct": ([i32, i32, i32, u32, ctypes.c_double, P(vp)], ctypes.c_int),
        "polar_code_free": ([vp], ctypes.c_int),
        "polar_code_query": ([vp, vp, vp], ctypes.c_int),
        "polar_trellis_pool": ([i32, i32, i32, u64, vp], ctypes.c_int),
        "polar_encode": ([vp, vp, vp, i64, vp], ctypes.c_int),
        "polar_info_bits": ([vp, vp, vp, i64, vp], ctypes.c_int),
        "bp_decode": ([vp, vp, i64, P(BPParamsC), vp, vp, vp, vp], ctypes.c_int),
        "pp_mt_bp_decode": ([vp, vp, i64, P(BPParamsC), P(PPParamsC), vp, vp, vp, vp],
                            ctypes.c_int),
        "pp_mt_bp_decode_ex": ([vp, vp, i64, P(BPParamsC), P(PPParamsC), vp, vp, vp, vp,
                                P(LaunchCfgC), vp], ctypes.c_int),
        "pp_mt_bp_decode_trace": ([vp, vp, i64, P(BPParamsC), P(PPParamsC), vp, vp, vp, vp, i32,
                                   vp], ctypes.c_int),
        "polar_classify_errors": ([vp, vp, vp, vp, vp, i32, i64, i32, vp, vp, vp], ctypes.c_int),
        "polar_batched_workspace_bytes": ([i64], sz),
        "pp_mt_bp_decode_batched": ([vp, i32, vp, vp, vp, i64, P(BPParamsC), P(PPParamsC),
                                     vp, vp, vp, vp, vp, sz, P(LaunchCfgC), vp], ctypes.c_int),
        "pp_mt_bp_decode_batched_noalloc": ([vp, i32, vp, vp, vp, i64, P(BPParamsC), P(PPParamsC),
                                             vp, vp, vp, vp, P(LaunchCfgC), vp], ctypes.c_int),
        "wbp_workspace_bytes": ([vp, i64, i32], sz),
        "wbp_forward": ([vp, vp, i64, vp, i32, P(PPParamsC), vp, vp, sz, vp], ctypes.c_int),
        "wbp_backward": ([vp, vp, i64, vp, i32, P(PPParamsC), vp, vp, vp, sz, vp],
                         ctypes.c_int),
        "polar_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "polar_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return _lib


def check(rc: int, where: str) -> None:
    if rc != PC_OK:
        raise PolarError(rc, where)
