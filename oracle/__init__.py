"""CPU oracle for PP-MT-BP polar decoding: ctypes shim over ``oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU library (``paper_1911_08868_amd``); neither imports the
other.  Every function is a thin marshalling layer; the arithmetic is in the
C file, which cites the passage of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# plain IEEE arithmetic: no contraction into fused multiply-add, no fast-math
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wno-unused-function"]


def build_library(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_library(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        c_i32, c_i64, c_u32, c_u64, c_d = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_double)
        vp = ctypes.c_void_p
        L.or_bhattacharyya.argtypes = [c_i32, c_d, vp]
        L.or_bhattacharyya.restype = ctypes.c_int
        L.or_construct.argtypes = [c_i32, c_i32, c_d, vp, vp, vp]
        L.or_construct.restype = ctypes.c_int
        L.or_crc_bits.argtypes = [vp, c_i64, c_i32, c_u32]
        L.or_crc_bits.restype = c_u32
        L.or_polar_transform.argtypes = [c_i32, vp, vp]
        L.or_polar_transform.restype = None
        L.or_encode.argtypes = [c_i32, c_i32, vp, c_i32, c_u32, vp, c_i64, vp, vp]
        L.or_encode.restype = ctypes.c_int
        L.or_splitmix64_next.argtypes = [P(c_u64)]
        L.or_splitmix64_next.restype = c_u64
        L.or_trellis_pool.argtypes = [c_i32, c_i32, c_i32, c_u64, vp]
        L.or_trellis_pool.restype = ctypes.c_int
        L.or_decode.argtypes = [c_i32, c_i32, vp, c_i32, c_u32, vp, c_i64, vp, vp, vp, vp, vp,
                                vp, c_i32]
        L.or_decode.restype = ctypes.c_int
        L.or_decode_trace.argtypes = [c_i32, c_i32, vp, c_i32, c_u32, vp, c_i64, vp, vp, vp, vp,
                                      vp, c_i32, c_i32]
        L.or_decode_trace.restype = ctypes.c_int
        L.or_noise_gauss.argtypes = [c_u64, c_i64, c_i32, c_i32]
        L.or_noise_gauss.restype = ctypes.c_float
        L.or_decision_key.argtypes = [c_i32]
        L.or_decision_key.restype = c_u64
        L.or_classify.argtypes = [c_i64, c_i32, vp, vp, vp, vp, vp, c_i32, vp, vp]
        L.or_classify.restype = ctypes.c_int
        L.or_wbp_forward.argtypes = [c_i32, c_i32, vp, vp, c_i64, vp, c_i32, vp, vp]
        L.or_wbp_forward.restype = ctypes.c_int
        L.or_wbp_backward.argtypes = [c_i32, c_i32, vp, vp, c_i64, vp, c_i32, vp, vp, vp, vp,
                                      vp]
        L.or_wbp_backward.restype = ctypes.c_int
        L.or_bp_run.argtypes = [c_i32, c_i32, vp, vp, vp, c_d, c_i32, c_i32, vp, vp]
        L.or_bp_run.restype = ctypes.c_int
        L.or_bp_continue.argtypes = [c_i32, c_i32, vp, c_d, c_i32, c_i32, vp, vp]
        L.or_bp_continue.restype = ctypes.c_int
        L.or_graph_encode.argtypes = [c_i32, vp, vp, vp]
        L.or_graph_encode.restype = ctypes.c_int
        L.or_alg1_trace.argtypes = [c_i32, c_i32, c_i32, c_i32, c_i32, c_u64, c_i32, vp, vp, vp,
                                    vp, vp]
        L.or_alg1_trace.restype = ctypes.c_int
        L.or_alg1_trace_r2.argtypes = [c_i32, c_i32, c_i32, c_u64, c_i32, vp, vp]
        L.or_alg1_trace_r2.restype = ctypes.c_int
        L.or_sizeof_params.restype = c_i32
        L.or_sizeof_wbp_params.restype = c_i32
        if L.or_sizeof_params() != ctypes.sizeof(_Params):
            raise RuntimeError("oracle parameter struct layout mismatch")
        if L.or_sizeof_wbp_params() != ctypes.sizeof(_WbpParams):
            raise RuntimeError("oracle weighted-BP parameter struct layout mismatch")
        _lib = L
    return _lib


class _Params(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("stop", ctypes.c_int32), ("it_min", ctypes.c_int32),
                ("pp_mode", ctypes.c_int32), ("k", ctypes.c_int32), ("T", ctypes.c_int32),
                ("Q", ctypes.c_int32), ("P_range", ctypes.c_int32), ("P_level", ctypes.c_int32),
                ("D", ctypes.c_int32), ("N_min", ctypes.c_int32),
                ("first_reset", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("fp32", ctypes.c_int32), ("exact_boxplus", ctypes.c_int32),
                ("noise_sigma", ctypes.c_float)]


class _WbpParams(ctypes.Structure):
    _fields_ = [("pp_mode", ctypes.c_int32), ("k", ctypes.c_int32), ("T_ev", ctypes.c_int32),
                ("Q", ctypes.c_int32), ("seed", ctypes.c_uint64), ("fp32", ctypes.c_int32)]


STOP_NONE, STOP_G, STOP_CRC = 0, 1, 2
PP_NONE, PP_LASTK, PP_FULL, PP_ALG1 = -1, 0, 1, 2
PP_ALG1_R2 = 3  # Algorithm 1 under the alternative reading R2 (blocks of the original graph)
PP_ALG1_ORIG = PP_ALG1_R2  # the library's name for the same mode


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class Code:
    """Polar code: length N, K information positions (CRC included)."""
    N: int
    K: int
    info_idx: np.ndarray  # int32 [K] ascending
    frozen: np.ndarray    # uint8 [N]
    crc_width: int = 0
    crc_poly: int = 0

    @property
    def n(self) -> int:
        return self.N.bit_length() - 1

    @property
    def K_msg(self) -> int:
        return self.K - self.crc_width


def bhattacharyya(N: int, lnz0: float) -> np.ndarray:
    out = np.zeros(N, np.float64)
    rc = lib().or_bhattacharyya(N, lnz0, _ptr(out))
    if rc:
        raise ValueError(f"or_bhattacharyya rc={rc}")
    return out


def construct(N: int, K: int, design_ebn0_db: float, crc_width: int = 0,
              crc_poly: int = 0) -> Code:
    info = np.zeros(K, np.int32)
    frozen = np.zeros(N, np.uint8)
    rc = lib().or_construct(N, K, float(design_ebn0_db), _ptr(info), _ptr(frozen), None)
    if rc:
        raise ValueError(f"or_construct rc={rc}")
    return Code(N, K, info, frozen, crc_width, crc_poly)


def construct_lnz(N: int, K: int, design_ebn0_db: float) -> np.ndarray:
    info = np.zeros(K, np.int32)
    lz = np.zeros(N, np.float64)
    rc = lib().or_construct(N, K, float(design_ebn0_db), _ptr(info), None, _ptr(lz))
    if rc:
        raise ValueError(f"or_construct rc={rc}")
    return lz


def crc(bits, width: int, poly: int) -> int:
    b = np.ascontiguousarray(np.asarray(bits, np.uint8))
    return int(lib().or_crc_bits(_ptr(b) if b.size else None, b.size, width, poly))


def polar_transform(u) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(u, np.uint8))
    x = np.zeros_like(u)
    lib().or_polar_transform(u.size, _ptr(u), _ptr(x))
    return x


def encode(code: Code, msg: np.ndarray):
    """msg uint8 [F, K_msg] -> (u [F, N], x [F, N])."""
    msg = np.ascontiguousarray(msg, np.uint8)
    F = msg.shape[0]
    u = np.zeros((F, code.N), np.uint8)
    x = np.zeros((F, code.N), np.uint8)
    rc = lib().or_encode(code.N, code.K, _ptr(code.info_idx), code.crc_width, code.crc_poly,
                         _ptr(msg), F, _ptr(u), _ptr(x))
    if rc:
        raise ValueError(f"or_encode rc={rc}")
    return u, x


def splitmix64_stream(seed: int, count: int) -> list[int]:
    st = ctypes.c_uint64(seed)
    return [int(lib().or_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def trellis_pool(n: int, k: int, Q: int, seed: int) -> np.ndarray:
    out = np.zeros((Q, n), np.int8)
    q = lib().or_trellis_pool(n, k, Q, seed, _ptr(out))
    if q < 0:
        raise ValueError(f"or_trellis_pool rc={q}")
    return out[:q].copy()


@dataclass
class DecodeParams:
    max_iter: int = 40
    alpha: float = 1.0
    stop: int = STOP_CRC
    it_min: int = 1
    pp_mode: int = PP_NONE
    k: int = 0
    T: int = 1
    Q: int = 1
    P_range: int = 2
    P_level: int = 1
    D: int = 1
    N_min: int = 1
    first_reset: int = 0
    seed: int = 0
    fp32: bool = True
    exact_boxplus: bool = False
    noise_sigma: float = 0.0

    def _c(self) -> _Params:
        return _Params(self.max_iter, self.alpha, self.stop, self.it_min, self.pp_mode, self.k,
                       self.T, self.Q, self.P_range, self.P_level, self.D, self.N_min,
                       self.first_reset, self.seed, int(self.fp32), int(self.exact_boxplus),
                       self.noise_sigma)


@dataclass
class DecodeResult:
    msg_hat: np.ndarray
    iters: np.ndarray
    ok: np.ndarray
    soft_u: np.ndarray | None = None
    state: np.ndarray | None = None


def decode(code: Code, llr: np.ndarray, params: DecodeParams, soft: bool = False,
           state: bool = False, threads: int = 1) -> DecodeResult:
    """llr float32 [F, N] -> hard message bits, iterations, check verdicts.

    soft=True also returns L at level n+1 after the final L sweep ([F, N]
    float64); state=True returns the final L and R arrays ([F, 2, n+1, N]).
    """
    llr = np.ascontiguousarray(llr, np.float32)
    F = llr.shape[0]
    assert llr.shape[1] == code.N
    msg = np.zeros((F, code.K_msg), np.uint8)
    it = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    su = np.zeros((F, code.N), np.float64) if soft else None
    st = np.zeros((F, 2, code.n + 1, code.N), np.float64) if state else None
    p = params._c()
    rc = lib().or_decode(code.N, code.K, _ptr(code.info_idx), code.crc_width, code.crc_poly,
                         _ptr(llr) if F else None, F, ctypes.byref(p), _ptr(msg) if F else None,
                         _ptr(it) if F else None, _ptr(ok) if F else None,
                         _ptr(su) if su is not None and F else None,
                         _ptr(st) if st is not None and F else None, threads)
    if rc:
        raise ValueError(f"or_decode rc={rc}")
    return DecodeResult(msg, it, ok, su, st)


CORRECT, FALSE_CONVERGED, OSCILLATION, UNCONVERGED = 0, 1, 2, 3


def decode_trace(code: Code, llr: np.ndarray, params: DecodeParams, H: int,
                 threads: int = 1):
    """``decode`` that also records the decision hash after every iteration.

    Returns (DecodeResult, hist uint64 [F, H]); the hash after iteration it
    (1-based) sits in column (it - 1) mod H; columns a frame did not reach
    stay 0."""
    llr = np.ascontiguousarray(llr, np.float32)
    F = llr.shape[0]
    assert llr.shape[1] == code.N
    msg = np.zeros((F, code.K_msg), np.uint8)
    it = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    hist = np.zeros((F, H), np.uint64)
    p = params._c()
    rc = lib().or_decode_trace(code.N, code.K, _ptr(code.info_idx), code.crc_width, code.crc_poly,
                               _ptr(llr) if F else None, F, ctypes.byref(p),
                               _ptr(msg) if F else None, _ptr(it) if F else None,
                               _ptr(ok) if F else None, _ptr(hist) if F else None, H, threads)
    if rc:
        raise ValueError(f"or_decode_trace rc={rc}")
    return DecodeResult(msg, it, ok), hist


def noise_gauss(seed: int, frame: int, e: int, j: int) -> float:
    return float(lib().or_noise_gauss(seed, frame, e, j))


def decision_key(j: int) -> int:
    return int(lib().or_decision_key(j))


def classify(msg_hat: np.ndarray, msg: np.ndarray, ok: np.ndarray, iters: np.ndarray,
             hist: np.ndarray):
    """Error class (CORRECT .. UNCONVERGED) and decision period of each frame."""
    msg_hat = np.ascontiguousarray(msg_hat, np.uint8)
    msg = np.ascontiguousarray(msg, np.uint8)
    ok = np.ascontiguousarray(ok, np.uint8)
    iters = np.ascontiguousarray(iters, np.int32)
    hist = np.ascontiguousarray(hist, np.uint64)
    F, K_msg = msg_hat.shape
    H = hist.shape[1]
    cls = np.zeros(F, np.uint8)
    per = np.zeros(F, np.int32)
    rc = lib().or_classify(F, K_msg, _ptr(msg_hat), _ptr(msg), _ptr(ok), _ptr(iters), _ptr(hist),
                           H, _ptr(cls), _ptr(per))
    if rc:
        raise ValueError(f"or_classify rc={rc}")
    return cls, per


@dataclass
class WbpParams:
    pp_mode: int = PP_NONE
    k: int = 0
    T_ev: int = 1
    Q: int = 1
    seed: int = 0
    fp32: bool = False

    def _c(self) -> _WbpParams:
        return _WbpParams(self.pp_mode, self.k, self.T_ev, self.Q, self.seed, int(self.fp32))


def wbp_forward(code: Code, llr: np.ndarray, w: np.ndarray, params: WbpParams) -> np.ndarray:
    """Weighted unrolled BP.  w float64 [T, n, 2, N] -> output LLRs [F, N]."""
    llr = np.ascontiguousarray(llr, np.float32)
    w = np.ascontiguousarray(w, np.float64)
    T = w.shape[0]
    assert w.shape == (T, code.n, 2, code.N)
    F = llr.shape[0]
    out = np.zeros((F, code.N), np.float64)
    p = params._c()
    rc = lib().or_wbp_forward(code.N, code.K, _ptr(code.info_idx), _ptr(llr), F, _ptr(w), T,
                              ctypes.byref(p), _ptr(out))
    if rc:
        raise ValueError(f"or_wbp_forward rc={rc}")
    return out


def wbp_backward(code: Code, llr: np.ndarray, w: np.ndarray, params: WbpParams,
                 grad_out: np.ndarray, want_llr_grad: bool = False, want_abs: bool = False):
    """Reverse mode of ``wbp_forward``: returns (grad_w [T,n,2,N], grad_llr or
    None), and with want_abs a third array: per weight entry, the sum over
    every path of the reverse computation of the magnitude of the path's
    product of derivatives (the scale of an FP32 adjoint's rounding error)."""
    llr = np.ascontiguousarray(llr, np.float32)
    w = np.ascontiguousarray(w, np.float64)
    g = np.ascontiguousarray(grad_out, np.float64)
    T = w.shape[0]
    F = llr.shape[0]
    gw = np.zeros_like(w)
    gl = np.zeros((F, code.N), np.float64) if want_llr_grad else None
    ga = np.zeros_like(w) if want_abs else None
    p = params._c()
    rc = lib().or_wbp_backward(code.N, code.K, _ptr(code.info_idx), _ptr(llr), F, _ptr(w), T,
                               ctypes.byref(p), _ptr(g), _ptr(gw),
                               _ptr(gl) if gl is not None else None,
                               _ptr(ga) if ga is not None else None)
    if rc:
        raise ValueError(f"or_wbp_backward rc={rc}")
    return (gw, gl, ga) if want_abs else (gw, gl)


def bp_run(llr: np.ndarray, frozen: np.ndarray, n_iter: int, order=None, alpha: float = 1.0,
           fp32: bool = True, exact: bool = False):
    """Plain BP for n_iter iterations on a fixed graph -> (L, R) [n+1, N].

    order: None (original graph), an [n] stage->bit list shared by all rows,
    or an [N, n] per-row table.
    """
    llr = np.ascontiguousarray(llr, np.float32).reshape(-1)
    N = llr.size
    n = N.bit_length() - 1
    if order is None:
        order = np.arange(n, dtype=np.int8)
    order = np.asarray(order, np.int8)
    if order.ndim == 1:
        order = np.tile(order, (N, 1))
    order = np.ascontiguousarray(order, np.int8)
    fr = np.ascontiguousarray(frozen, np.uint8)
    L = np.zeros((n + 1, N), np.float64)
    R = np.zeros((n + 1, N), np.float64)
    rc = lib().or_bp_run(N, n_iter, _ptr(order), _ptr(llr), _ptr(fr), alpha, int(fp32),
                         int(exact), _ptr(L), _ptr(R))
    if rc:
        raise ValueError(f"or_bp_run rc={rc}")
    return L, R


def graph_encode(order: np.ndarray, u) -> np.ndarray:
    """Encode u through the graph with per-row stage order [N, n]."""
    order = np.ascontiguousarray(order, np.int8)
    u = np.ascontiguousarray(np.asarray(u, np.uint8))
    x = np.zeros_like(u)
    rc = lib().or_graph_encode(u.size, _ptr(order), _ptr(u), _ptr(x))
    if rc:
        raise ValueError(f"or_graph_encode rc={rc}")
    return x


def alg1_trace(N: int, P_range: int, P_level: int, D: int, N_min: int, seed: int,
               n_events: int, want_draws: bool = False):
    """Schedules and counters after each of n_events Algorithm-1 events; with
    want_draws also the accepted draw of each event, int32 [n_events, 4 + n]:
    rho_range, x, m, block, then the new bits of stages rho_level..m
    (rho_range = 0 for a skipped event)."""
    n = N.bit_length() - 1
    ords = np.zeros((n_events, N, n), np.int8)
    nz = np.zeros(n_events, np.int32)
    add = np.zeros(n_events, np.int32)
    zc = np.zeros(n_events, np.int32)
    dr = np.zeros((n_events, 4 + n), np.int32)
    rc = lib().or_alg1_trace(N, P_range, P_level, D, N_min, seed, n_events, _ptr(ords),
                             _ptr(nz), _ptr(add), _ptr(zc), _ptr(dr))
    if rc:
        raise ValueError(f"or_alg1_trace rc={rc}")
    return (ords, nz, add, zc, dr) if want_draws else (ords, nz, add, zc)


def alg1_trace_r2(N: int, P_range: int, P_level: int, seed: int, n_events: int):
    """Schedules and N_zero after each of n_events events under reading R2."""
    n = N.bit_length() - 1
    ords = np.zeros((n_events, N, n), np.int8)
    nz = np.zeros(n_events, np.int32)
    rc = lib().or_alg1_trace_r2(N, P_range, P_level, seed, n_events, _ptr(ords), _ptr(nz))
    if rc:
        raise ValueError(f"or_alg1_trace_r2 rc={rc}")
    return ords, nz


def bp_continue(L: np.ndarray, R: np.ndarray, n_iter: int, order=None, alpha: float = 1.0,
                fp32: bool = True, exact: bool = False):
    """Run n_iter more plain BP iterations from state (L, R) [n+1, N]; returns copies."""
    L = np.ascontiguousarray(L, np.float64).copy()
    R = np.ascontiguousarray(R, np.float64).copy()
    N = L.shape[1]
    n = N.bit_length() - 1
    if order is None:
        order = np.arange(n, dtype=np.int8)
    order = np.asarray(order, np.int8)
    if order.ndim == 1:
        order = np.tile(order, (N, 1))
    order = np.ascontiguousarray(order, np.int8)
    rc = lib().or_bp_continue(N, n_iter, _ptr(order), alpha, int(fp32), int(exact), _ptr(L),
                              _ptr(R))
    if rc:
        raise ValueError(f"or_bp_continue rc={rc}")
    return L, R
