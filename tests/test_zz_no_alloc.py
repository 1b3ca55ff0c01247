"""The allocation-free batched entry point (pp_mt_bp_decode_batched_noalloc)
against pp_mt_bp_decode_batched with a caller workspace, through the C ABI:
two calls in a row on the shared scratch, the second with fewer frames, each
equal to the workspace call bit for bit (decided bits, iteration counts,
verdicts); the size limit and the empty call."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SPECS = [(64, 40), (128, 43), (256, 171), (512, 256), (1024, 512), (1024, 768)]


@pytest.fixture(scope="module")
def pbp():
    import torch
    assert torch.cuda.is_available()
    import paper_1911_08868_amd as m
    return m


def _frames(pbp, codes, F, seed):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    cid = torch.randint(0, len(codes), (F,), generator=gen, device="cuda", dtype=torch.int32)
    Ns = torch.tensor([c.N for c in codes], device="cuda")
    Ks = torch.tensor([c.K_msg for c in codes], device="cuda")
    n_f, k_f = Ns[cid.long()], Ks[cid.long()]
    llr_off = torch.cumsum(n_f, 0) - n_f
    bits_off = torch.cumsum(k_f, 0) - k_f
    pool = torch.zeros(int(n_f.sum().item()), dtype=torch.float32, device="cuda")
    for i, c in enumerate(codes):
        idx = torch.nonzero(cid == i).flatten()
        if idx.numel() == 0:
            continue
        m = torch.randint(0, 2, (idx.numel(), c.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
        ebn0 = torch.rand(idx.numel(), generator=gen, device="cuda", dtype=torch.float64) * 3.0 + 1.0
        llr = synth.awgn_llr_torch(pbp.encode(c, m), ebn0, c.K_msg, gen)
        rows = llr_off[idx].view(-1, 1) + torch.arange(c.N, device="cuda").view(1, -1)
        pool[rows.flatten()] = llr.flatten()
    return cid, llr_off.to(torch.int64), bits_off.to(torch.int64), pool, int(k_f.sum().item())


def _call(pbp, codes, frames, bp, pp, noalloc):
    import torch
    cid, llr_off, bits_off, pool, nbits = frames
    F = cid.numel()
    bits = torch.full((max(nbits, 1),), 7, dtype=torch.uint8, device="cuda")
    iters = torch.full((max(F, 1),), -1, dtype=torch.int32, device="cuda")
    ok = torch.full((max(F, 1),), 9, dtype=torch.uint8, device="cuda")
    handles = (ctypes.c_void_p * len(codes))(*[c.handle.value for c in codes])
    bpc, ppc = bp.c(), pp.c()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    args = (handles, len(codes), P(cid.data_ptr()), P(llr_off.data_ptr()), P(pool.data_ptr()), F,
            ctypes.byref(bpc), ctypes.byref(ppc), P(bits.data_ptr()), P(bits_off.data_ptr()),
            P(iters.data_ptr()), P(ok.data_ptr()))
    if noalloc:
        rc = pbp.lib().pp_mt_bp_decode_batched_noalloc(*args, None, stream)
    else:
        ws = torch.empty(pbp.batched_workspace_bytes(F), dtype=torch.uint8, device="cuda")
        rc = pbp.lib().pp_mt_bp_decode_batched(*args, P(ws.data_ptr()), ws.numel(), None, stream)
    assert rc == 0, pbp.lib().polar_last_error()
    torch.cuda.synchronize()
    return bits.cpu().numpy(), iters.cpu().numpy(), ok.cpu().numpy()


@pytest.mark.parametrize("pp_on", [True, False])
def test_noalloc_equals_workspace_call(pbp, pp_on):
    codes = [pbp.Code(N, K, 16, 0x1021, 2.5) for N, K in SPECS]
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    pp = (pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=3) if pp_on
          else pbp.PPParams())
    for F, seed in ((6000, 11), (1500, 12)):      # the second call is smaller
        fr = _frames(pbp, codes, F, seed + int(pp_on))
        ref = _call(pbp, codes, fr, bp, pp, noalloc=False)
        got = _call(pbp, codes, fr, bp, pp, noalloc=True)
        for r, g, what in zip(ref, got, ("bits", "iterations", "verdicts")):
            assert np.array_equal(r, g), f"F={F}: {what} differ"
        assert (ref[1] >= 1).all() and (ref[1] <= 200).all()


def test_noalloc_limits(pbp):
    import torch
    codes = [pbp.Code(256, 128, 16, 0x1021, 2.5)]
    bp = pbp.BPParams(max_iter=20, stop=pbp.STOP_CRC, it_min=3)
    handles = (ctypes.c_void_p * 1)(codes[0].handle.value)
    bpc, ppc = bp.c(), pbp.PPParams().c()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dummy = torch.zeros(16, dtype=torch.int64, device="cuda")
    P = ctypes.c_void_p(dummy.data_ptr())
    L = pbp.lib()
    # more frames than the scratch holds: rejected before any launch
    rc = L.pp_mt_bp_decode_batched_noalloc(handles, 1, P, P, P, (1 << 20) + 1, ctypes.byref(bpc),
                                           ctypes.byref(ppc), P, P, P, P, None, stream)
    assert rc == pbp.PC_EINVAL and b"1048576" in L.polar_last_error()
    # no frames: a no-op
    rc = L.pp_mt_bp_decode_batched_noalloc(handles, 1, None, None, None, 0, ctypes.byref(bpc),
                                           ctypes.byref(ppc), None, None, None, None, None, stream)
    assert rc == 0
