"""MI355X-native PP-MT-BP polar decoding (arXiv 1911.08868).

Thin Python binding over the C ABI of ``libpolarbp.so`` (see
``include/polarbp.h``).  The functions here only marshal arguments: device
buffers are torch tensors on a ROCm device, the stream is torch's current
stream, and every step of decoding runs in the library's HIP kernels.  There
is no CPU fallback: if the library is missing, importing the binding's
functions raises.
"""
from __future__ import annotations

from ._lib import (PolarError, PC_OK, PC_EINVAL, PC_ENOTSUP, PC_EHIP, PC_ENOMEM,
                   STOP_NONE, STOP_G, STOP_CRC, PP_NONE, PP_LASTK, PP_FULL, PP_ALG1, PP_ALG1_ORIG,
                   ERR_CORRECT, ERR_FALSE_CONVERGED, ERR_OSCILLATION, ERR_UNCONVERGED,
                   CHECK_MINSUM, CHECK_EXACT, lib, library_path)
from .api import (Code, BPParams, PPParams, LaunchCfg, trellis_pool, encode, info_bits, bp_decode,
                  pp_mt_bp_decode, pp_mt_bp_decode_trace, classify_errors, decode_batched,
                  batched_workspace_bytes, wbp_workspace_bytes, wbp_forward, wbp_backward)

__all__ = [
    "PolarError", "PC_OK", "PC_EINVAL", "PC_ENOTSUP", "PC_EHIP", "PC_ENOMEM",
    "STOP_NONE", "STOP_G", "STOP_CRC", "PP_NONE", "PP_LASTK", "PP_FULL", "PP_ALG1", "PP_ALG1_ORIG",
    "lib", "library_path", "Code", "BPParams", "PPParams", "LaunchCfg", "trellis_pool",
    "encode", "info_bits", "bp_decode", "pp_mt_bp_decode", "decode_batched", "batched_workspace_bytes",
    "wbp_workspace_bytes", "wbp_forward", "wbp_backward", "pp_mt_bp_decode_trace",
    "classify_errors", "CHECK_MINSUM", "CHECK_EXACT", "ERR_CORRECT", "ERR_FALSE_CONVERGED", "ERR_OSCILLATION", "ERR_UNCONVERGED",
]

from . import wbp  # noqa: E402  (torch.autograd wrapper of the weighted kernels)
from . import batched, tune  # noqa: E402,F401
