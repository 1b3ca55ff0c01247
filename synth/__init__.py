"""Seeded synthetic inputs: message bits, Eb/N0 draws and BPSK-AWGN channel LLRs.

This module holds the experiment's channel model (Sec. IV: AWGN, with the
energy per bit counted over the message bits only) and nothing of the
decoding method: no code construction, encoding, CRC or BP arithmetic.  It is
the one module that both the oracle-side tests and the GPU-side tests and
benchmark draw inputs from.  Codeword bits are an input here; callers encode
them with whichever implementation they are testing against.

QPSK over AWGN, as simulated in the paper, is two independent BPSK
dimensions at the same Eb/N0, so BPSK frames are used throughout.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    # Philox is counter based: (seed, stream) give independent reproducible streams
    return np.random.Generator(np.random.Philox(key=[seed & 0xFFFFFFFFFFFFFFFF,
                                                     stream & 0xFFFFFFFFFFFFFFFF]))


def message_bits(seed: int, F: int, k_msg: int, all_zero: bool = False,
                 stream: int = 1) -> np.ndarray:
    """uint8 [F, k_msg]: uniform random bits, or all zeros."""
    if all_zero:
        return np.zeros((F, k_msg), np.uint8)
    return _rng(seed, stream).integers(0, 2, size=(F, k_msg), dtype=np.uint8)


def ebn0_uniform(seed: int, F: int, lo_db: float, hi_db: float, stream: int = 3) -> np.ndarray:
    """float64 [F]: per-frame Eb/N0 in dB, uniform on [lo_db, hi_db]."""
    return _rng(seed, stream).uniform(lo_db, hi_db, size=F)


def noise_sigma2(ebn0_db, n: int, k_msg: int):
    """Noise variance per real dimension for unit-energy BPSK symbols.

    Es = R_e * Eb with R_e = k_msg / N (CRC bits excluded from the energy per
    information bit), N0 = 2 sigma^2.
    """
    r_e = k_msg / n
    return 1.0 / (2.0 * r_e * np.power(10.0, np.asarray(ebn0_db, np.float64) / 10.0))


def awgn_llr(x: np.ndarray, ebn0_db, k_msg: int, seed: int, stream: int = 2,
             noiseless: bool = False) -> np.ndarray:
    """Channel LLRs for codeword bits x (uint8 [F, N]).

    Bit 0 -> +1, bit 1 -> -1; y = s + sigma z with z ~ N(0,1) in float64;
    LLR = 2 y / sigma^2, rounded once to float32 (positive favours bit 0).
    ebn0_db is a scalar or a per-frame array.
    """
    x = np.asarray(x, np.uint8)
    F, N = x.shape
    s = 1.0 - 2.0 * x.astype(np.float64)
    sig2 = noise_sigma2(ebn0_db, N, k_msg)
    sig2 = np.broadcast_to(np.asarray(sig2, np.float64).reshape(-1, 1) if np.ndim(sig2)
                           else np.asarray(sig2, np.float64), (F, 1))
    if noiseless:
        y = s
    else:
        z = _rng(seed, stream).standard_normal(size=(F, N))
        y = s + np.sqrt(sig2) * z
    return (2.0 * y / sig2).astype(np.float32)


def awgn_llr_torch(x, ebn0_db, k_msg: int, generator, out=None):
    """Same channel as ``awgn_llr`` on a torch device tensor x (uint8 [F, N]).

    Used to fill large benchmark batches directly in device memory; the
    noise comes from the given torch.Generator, in float32.
    """
    import torch
    F, N = x.shape
    s = 1.0 - 2.0 * x.to(torch.float32)
    e = torch.as_tensor(ebn0_db, dtype=torch.float64, device=x.device)
    sig2 = (1.0 / (2.0 * (k_msg / N) * torch.pow(10.0, e / 10.0))).to(torch.float32)
    if sig2.dim() == 1:
        sig2 = sig2.view(-1, 1)
    z = torch.randn((F, N), generator=generator, device=x.device, dtype=torch.float32)
    y = s + torch.sqrt(sig2) * z
    llr = 2.0 * y / sig2
    if out is not None:
        out.copy_(llr)
        return out
    return llr
