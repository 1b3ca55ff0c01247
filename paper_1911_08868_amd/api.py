"""Python wrappers with the names of the C ABI (argument marshalling only).

Device buffers are torch tensors on the code's device; results are written
into caller-provided tensors or freshly allocated ones, on torch's current
stream.  Nothing here computes any part of the decoder.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from ._lib import (BPParamsC, LaunchCfgC, PPParamsC, PolarError, PP_ALG1, PP_FULL,  # noqa: F401
                   PP_LASTK, PP_NONE, STOP_CRC, STOP_G, STOP_NONE, CHECK_MINSUM, CHECK_EXACT,
                   check, lib)


def _torch():
    import torch
    return torch


def _stream(device=None):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _need(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class BPParams:
    max_iter: int = 200
    alpha: float = 1.0
    stop: int = STOP_CRC
    it_min: int = 1
    check: int = CHECK_MINSUM

    def c(self) -> BPParamsC:
        return BPParamsC(self.max_iter, self.alpha, self.stop, self.it_min, self.check)


@dataclass
class PPParams:
    mode: int = PP_NONE
    k: int = 0
    period_T: int = 10
    pool_Q: int = 8
    P_range: int = 0
    P_level: int = 0
    D: int = 0
    N_min: int = 0
    first_reset: int = 0
    seed: int = 0
    noise_sigma: float = 0.0

    def c(self) -> PPParamsC:
        return PPParamsC(self.mode, self.k, self.period_T, self.pool_Q, self.P_range,
                         self.P_level, self.D, self.N_min, self.first_reset, self.seed,
                         self.noise_sigma)


@dataclass
class LaunchCfg:
    rho: int = 0
    slots: int = 0
    grid: int = 0

    def c(self) -> LaunchCfgC:
        return LaunchCfgC(self.rho, self.slots, self.grid)


class Code:
    """A polar code on the current device (``polar_construct``)."""

    def __init__(self, N: int, K: int, crc_width: int = 0, crc_poly: int = 0,
                 design_ebn0_db: float = 2.5):
        h = ctypes.c_void_p()
        check(lib().polar_construct(N, K, crc_width, crc_poly, float(design_ebn0_db),
                                    ctypes.byref(h)), "polar_construct")
        self._h = h
        self.N, self.K, self.crc_width, self.crc_poly = N, K, crc_width, crc_poly
        self.n = N.bit_length() - 1
        self.K_msg = K - crc_width
        info = np.zeros(K, np.int32)
        frozen = np.zeros(N, np.uint8)
        check(lib().polar_code_query(h, info.ctypes.data_as(ctypes.c_void_p),
                                     frozen.ctypes.data_as(ctypes.c_void_p)), "polar_code_query")
        self.info_idx, self.frozen = info, frozen

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().polar_code_free(h)
            except Exception:
                pass
            self._h = None


def trellis_pool(n: int, k: int, Q: int, seed: int) -> np.ndarray:
    out = np.zeros((Q, n), np.int8)
    q = lib().polar_trellis_pool(n, k, Q, seed, out.ctypes.data_as(ctypes.c_void_p))
    if q < 0:
        check(q, "polar_trellis_pool")
    return out[:q].copy()


def encode(code: Code, msg, out=None):
    """msg uint8 [F, K_msg] on the device -> codewords uint8 [F, N]."""
    torch = _torch()
    F = msg.shape[0]
    _need(msg, torch.uint8, (F, code.K_msg), "msg")
    if out is None:
        out = torch.empty((F, code.N), dtype=torch.uint8, device=msg.device)
    _need(out, torch.uint8, (F, code.N), "out")
    check(lib().polar_encode(code.handle, _ptr(msg), _ptr(out), F, _stream(msg.device)),
          "polar_encode")
    return out


def info_bits(code: Code, msg, out=None):
    """msg uint8 [F, K_msg] on the device -> u on the information rows,
    uint8 [F, K] (the message, then its CRC), ``polar_info_bits``."""
    torch = _torch()
    F = msg.shape[0]
    _need(msg, torch.uint8, (F, code.K_msg), "msg")
    if out is None:
        out = torch.empty((F, code.K), dtype=torch.uint8, device=msg.device)
    _need(out, torch.uint8, (F, code.K), "out")
    check(lib().polar_info_bits(code.handle, _ptr(msg), _ptr(out), F, _stream(msg.device)),
          "polar_info_bits")
    return out


def _decode(code, llr, bp, pp, soft, cfg, out):
    torch = _torch()
    F = llr.shape[0]
    _need(llr, torch.float32, (F, code.N), "llr")
    dev = llr.device
    if out is None:
        out = (torch.empty((F, code.K_msg), dtype=torch.uint8, device=dev),
               torch.empty(F, dtype=torch.int32, device=dev),
               torch.empty(F, dtype=torch.uint8, device=dev))
    msg, iters, ok = out
    _need(msg, torch.uint8, (F, code.K_msg), "msg_hat")
    if iters is not None:
        _need(iters, torch.int32, (F,), "iters")
    if ok is not None:
        _need(ok, torch.uint8, (F,), "ok")
    soft_t = None
    if soft:
        soft_t = torch.empty((F, code.N), dtype=torch.float32, device=dev)
    bpc = bp.c()
    ppc = (pp or PPParams()).c()
    cfgc = cfg.c() if cfg is not None else None
    rc = lib().pp_mt_bp_decode_ex(code.handle, _ptr(llr), F, ctypes.byref(bpc), ctypes.byref(ppc),
                                  _ptr(msg), _ptr(iters), _ptr(ok), _ptr(soft_t),
                                  ctypes.byref(cfgc) if cfgc is not None else None,
                                  _stream(dev))
    check(rc, "pp_mt_bp_decode_ex")
    return (msg, iters, ok, soft_t) if soft else (msg, iters, ok)


def bp_decode(code: Code, llr, bp: BPParams, out=None, soft: bool = False,
              cfg: LaunchCfg | None = None):
    """Standard BP.  Returns (msg_hat uint8 [F,K_msg], iters int32 [F], ok uint8 [F])."""
    return _decode(code, llr, bp, None, soft, cfg, out)


def pp_mt_bp_decode(code: Code, llr, bp: BPParams, pp: PPParams, out=None, soft: bool = False,
                    cfg: LaunchCfg | None = None):
    """Partially permuted multi-trellis BP; same outputs as ``bp_decode``."""
    return _decode(code, llr, bp, pp, soft, cfg, out)


def pp_mt_bp_decode_trace(code: Code, llr, bp: BPParams, pp: PPParams | None, H: int = 32):
    """Decode and record the decision hash after every iteration (error
    classes, Sec. II-C).  Returns (msg_hat, iters, ok, hist [F, H]); hist
    holds the 64-bit hashes in an int64 tensor (same bits; view the host copy
    as uint64); the hash after iteration it (1-based) is at column
    (it - 1) mod H, columns a frame did not reach hold 0."""
    torch = _torch()
    F = llr.shape[0]
    _need(llr, torch.float32, (F, code.N), "llr")
    dev = llr.device
    msg = torch.empty((F, code.K_msg), dtype=torch.uint8, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev)
    ok = torch.empty(F, dtype=torch.uint8, device=dev)
    hist = torch.zeros((F, H), dtype=torch.int64, device=dev)
    bpc = bp.c()
    ppc = (pp or PPParams()).c()
    check(lib().pp_mt_bp_decode_trace(code.handle, _ptr(llr), F, ctypes.byref(bpc),
                                      ctypes.byref(ppc), _ptr(msg), _ptr(iters), _ptr(ok),
                                      _ptr(hist), H, _stream(dev)), "pp_mt_bp_decode_trace")
    return msg, iters, ok, hist


def classify_errors(msg_hat, msg, ok, iters, hist):
    """Error class (ERR_*) and decision period of each frame from a trace
    decode's outputs and the transmitted messages (all device tensors)."""
    torch = _torch()
    F, K_msg = msg_hat.shape
    H = hist.shape[1]
    _need(msg_hat, torch.uint8, (F, K_msg), "msg_hat")
    _need(msg, torch.uint8, (F, K_msg), "msg")
    _need(ok, torch.uint8, (F,), "ok")
    _need(iters, torch.int32, (F,), "iters")
    _need(hist, torch.int64, (F, H), "hist")
    cls = torch.empty(F, dtype=torch.uint8, device=msg_hat.device)
    per = torch.empty(F, dtype=torch.int32, device=msg_hat.device)
    check(lib().polar_classify_errors(_ptr(msg_hat), _ptr(msg), _ptr(ok), _ptr(iters), _ptr(hist),
                                      H, F, K_msg, _ptr(cls), _ptr(per), _stream(msg_hat.device)),
          "polar_classify_errors")
    return cls, per


def batched_workspace_bytes(F: int) -> int:
    return int(lib().polar_batched_workspace_bytes(F))


def decode_batched(codes, code_id, llr_off, llr_pool, bp: BPParams, pp: PPParams | None,
                   bits_pool, bits_off, iters=None, ok=None, workspace=None,
                   cfg: LaunchCfg | None = None):
    """Mixed-length batch through the persistent queue kernel (see the C header).

    Returns the workspace tensor used (allocate it once and pass it back for
    repeated or graph-captured rounds)."""
    torch = _torch()
    F = code_id.shape[0]
    dev = llr_pool.device
    _need(code_id, torch.int32, (F,), "code_id")
    _need(llr_off, torch.int64, (F,), "llr_off")
    _need(bits_off, torch.int64, (F,), "bits_off")
    if iters is not None:
        _need(iters, torch.int32, (F,), "iters")
    if ok is not None:
        _need(ok, torch.uint8, (F,), "ok")
    ws_bytes = batched_workspace_bytes(F)
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    handles = (ctypes.c_void_p * len(codes))(*[c.handle.value for c in codes])
    bpc = bp.c()
    ppc = (pp or PPParams()).c()
    cfgc = cfg.c() if cfg is not None else None
    rc = lib().pp_mt_bp_decode_batched(handles, len(codes), _ptr(code_id), _ptr(llr_off),
                                       _ptr(llr_pool), F, ctypes.byref(bpc), ctypes.byref(ppc),
                                       _ptr(bits_pool), _ptr(bits_off), _ptr(iters), _ptr(ok),
                                       _ptr(workspace), workspace.numel(),
                                       ctypes.byref(cfgc) if cfgc is not None else None,
                                       _stream(dev))
    check(rc, "pp_mt_bp_decode_batched")
    return workspace


def wbp_workspace_bytes(code: Code, F: int, T: int) -> int:
    return int(lib().wbp_workspace_bytes(code.handle, F, T))


def wbp_forward(code: Code, llr, w, pp: PPParams | None, out, workspace):
    """workspace=None: forward pass alone, no checkpoints (no backward may follow)."""
    torch = _torch()
    F = llr.shape[0]
    T = w.shape[0]
    _need(llr, torch.float32, (F, code.N), "llr")
    _need(w, torch.float32, (T, code.n, 2, code.N), "w")
    _need(out, torch.float32, (F, code.N), "out")
    ppc = pp.c() if pp is not None else None
    rc = lib().wbp_forward(code.handle, _ptr(llr), F, _ptr(w), T,
                           ctypes.byref(ppc) if ppc is not None else None, _ptr(out),
                           _ptr(workspace) if workspace is not None else None,
                           workspace.numel() * workspace.element_size() if workspace is not None else 0,
                           _stream(llr.device))
    check(rc, "wbp_forward")
    return out


def wbp_backward(code: Code, llr, w, pp: PPParams | None, grad_out, grad_w, workspace):
    torch = _torch()
    F = llr.shape[0]
    T = w.shape[0]
    _need(grad_out, torch.float32, (F, code.N), "grad_out")
    _need(grad_w, torch.float32, (T, code.n, 2, code.N), "grad_w")
    ppc = pp.c() if pp is not None else None
    rc = lib().wbp_backward(code.handle, _ptr(llr), F, _ptr(w), T,
                            ctypes.byref(ppc) if ppc is not None else None, _ptr(grad_out),
                            _ptr(grad_w), _ptr(workspace),
                            workspace.numel() * workspace.element_size(), _stream(llr.device))
    check(rc, "wbp_backward")
    return grad_w
