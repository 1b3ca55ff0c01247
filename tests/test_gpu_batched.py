"""GPU parity of the mixed-length persistent batched decoder against the oracle
(every frame decoded by the oracle with its own code), launch shapes that
force many queue refills and bucket changes, and HIP-graph replays checked
against eager runs."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SPECS = [(64, 24), (64, 40), (128, 43), (128, 96), (256, 85), (256, 171), (512, 256),
         (512, 384), (1024, 256), (1024, 768)]


@pytest.fixture(scope="module")
def pbp():
    import torch
    assert torch.cuda.is_available()
    import paper_1911_08868_amd as m
    return m


def _stream(orc, pbp, F, seed, specs=SPECS):
    """Frames of mixed codes built on the host with the oracle encoder."""
    import torch
    rng = np.random.default_rng(seed)
    ocodes = [orc.construct(N, K, 2.5, 16, 0x1021) for N, K in specs]
    gcodes = [pbp.Code(N, K, 16, 0x1021, 2.5) for N, K in specs]
    for o, g in zip(ocodes, gcodes):
        assert np.array_equal(o.info_idx, g.info_idx)
    cid = rng.integers(0, len(specs), F)
    snr = rng.uniform(1.0, 4.0, F)
    llr_off = np.zeros(F, np.int64)
    bits_off = np.zeros(F, np.int64)
    pos = bpos = 0
    frames = []
    for f in range(F):
        c = ocodes[cid[f]]
        llr_off[f], bits_off[f] = pos, bpos
        pos += c.N
        bpos += c.K_msg
    pool = np.zeros(pos, np.float32)
    msgs = {}
    for ci, c in enumerate(ocodes):
        idx = np.nonzero(cid == ci)[0]
        if idx.size == 0:
            continue
        m = synth.message_bits(seed * 100 + ci, idx.size, c.K_msg)
        _, x = orc.encode(c, m)
        l = synth.awgn_llr(x, snr[idx], c.K_msg, seed=seed * 100 + ci)
        for t, f in enumerate(idx):
            pool[llr_off[f]:llr_off[f] + c.N] = l[t]
        msgs[ci] = (idx, m, l)
    dev = dict(code_id=torch.from_numpy(cid.astype(np.int32)).cuda(),
               llr_off=torch.from_numpy(llr_off).cuda(),
               bits_off=torch.from_numpy(bits_off).cuda(),
               llr_pool=torch.from_numpy(pool).cuda(),
               bits_pool=torch.zeros(bpos, dtype=torch.uint8, device="cuda"),
               iters=torch.zeros(F, dtype=torch.int32, device="cuda"),
               ok=torch.zeros(F, dtype=torch.uint8, device="cuda"))
    return ocodes, gcodes, cid, bits_off, msgs, dev


def _oracle(orc, ocodes, msgs, pp_on, max_iter=200):
    out = {}
    for ci, (idx, m, l) in msgs.items():
        c = ocodes[ci]
        k = min(4, c.n - 1)
        p = orc.DecodeParams(max_iter=max_iter, stop=orc.STOP_CRC, it_min=3,
                             pp_mode=orc.PP_LASTK if pp_on else orc.PP_NONE, k=k if pp_on else 0,
                             T=10, Q=8, seed=9)
        out[ci] = orc.decode(c, l, p, threads=8)
    return out


def _check(ocodes, cid, bits_off, msgs, ref, dev):
    bits = dev["bits_pool"].cpu().numpy()
    iters = dev["iters"].cpu().numpy()
    ok = dev["ok"].cpu().numpy()
    for ci, (idx, m, l) in msgs.items():
        c = ocodes[ci]
        r = ref[ci]
        got = np.stack([bits[bits_off[f]:bits_off[f] + c.K_msg] for f in idx])
        assert np.array_equal(got, r.msg_hat), f"code {ci} bits"
        assert np.array_equal(iters[idx], r.iters), f"code {ci} iterations"
        assert np.array_equal(ok[idx], r.ok), f"code {ci} verdicts"


@pytest.mark.parametrize("pp_on", [True, False])
@pytest.mark.parametrize("rho,slots,grid", [(0, 1, 0), (0, 2, 0), (0, 1, 2), (2, 1, 0),
                                            (2, 2, 0), (3, 1, 0), (2, 1, 1), (2, 1, 3),
                                            (3, 2, 5)])
def test_batched_parity(orc, pbp, pp_on, rho, slots, grid):
    import torch
    ocodes, gcodes, cid, bits_off, msgs, dev = _stream(orc, pbp, 400, seed=rho * 7 + slots + grid)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=9) if pp_on else None
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    pbp.decode_batched(gcodes, dev["code_id"], dev["llr_off"], dev["llr_pool"], bp, pp,
                       dev["bits_pool"], dev["bits_off"], dev["iters"], dev["ok"],
                       cfg=pbp.LaunchCfg(rho, slots, grid))
    torch.cuda.synchronize()
    _check(ocodes, cid, bits_off, msgs, _oracle(orc, ocodes, msgs, pp_on), dev)


def test_batched_single_length_and_empty_buckets(orc, pbp):
    import torch
    specs = [(256, 128), (256, 200)]
    ocodes, gcodes, cid, bits_off, msgs, dev = _stream(orc, pbp, 150, seed=3, specs=specs)
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=9)
    pbp.decode_batched(gcodes, dev["code_id"], dev["llr_off"], dev["llr_pool"], bp, pp,
                       dev["bits_pool"], dev["bits_off"], dev["iters"], dev["ok"])
    torch.cuda.synchronize()
    _check(ocodes, cid, bits_off, msgs, _oracle(orc, ocodes, msgs, True), dev)


def test_batched_graph_replays(orc, pbp):
    """Capture one round, replay it on three different frame sets with eager
    work and synchronisation between replays; each replay must equal an eager
    run on the same data."""
    import torch
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=9)
    ocodes, gcodes, cid, bits_off, msgs, dev = _stream(orc, pbp, 300, seed=21)
    ws = torch.empty(pbp.batched_workspace_bytes(300), dtype=torch.uint8, device="cuda")
    call = lambda: pbp.decode_batched(gcodes, dev["code_id"], dev["llr_off"], dev["llr_pool"], bp,
                                      pp, dev["bits_pool"], dev["bits_off"], dev["iters"],
                                      dev["ok"], workspace=ws)
    call()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    base_pool = dev["llr_pool"].clone()
    for rep in range(3):
        # new frame data: flip the sign pattern of a random subset and rescale
        scale = torch.from_numpy(rng.uniform(0.6, 1.4, base_pool.numel()).astype(np.float32)).cuda()
        dev["llr_pool"].copy_(base_pool * scale)
        dev["bits_pool"].zero_()
        dev["iters"].zero_()
        g.replay()
        torch.cuda.synchronize()
        got = (dev["bits_pool"].clone(), dev["iters"].clone(), dev["ok"].clone())
        dev["bits_pool"].zero_()
        dev["iters"].fill_(-1)
        call()
        torch.cuda.synchronize()
        assert torch.equal(got[0], dev["bits_pool"]), f"replay {rep} bits"
        assert torch.equal(got[1], dev["iters"]), f"replay {rep} iterations"
        assert torch.equal(got[2], dev["ok"]), f"replay {rep} verdicts"
        _ = (base_pool * 2).sum().item()  # eager work between replays


def test_batched_rejects(pbp):
    import torch
    bp = pbp.BPParams(max_iter=10, stop=pbp.STOP_CRC)
    small = pbp.Code(32, 20, 16, 0x1021)
    z = torch.zeros(4, dtype=torch.int32, device="cuda")
    o = torch.zeros(4, dtype=torch.int64, device="cuda")
    pool = torch.zeros(4096, dtype=torch.float32, device="cuda")
    bits = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(pbp.PolarError):
        pbp.decode_batched([small], z, o, pool, bp, None, bits, o)
    c = pbp.Code(256, 128, 16, 0x1021)
    with pytest.raises(pbp.PolarError):
        pbp.decode_batched([c], z, o, pool, bp, pbp.PPParams(mode=pbp.PP_LASTK, k=3), bits, o)
    with pytest.raises(pbp.PolarError):
        pbp.decode_batched([c], z, o, pool, bp, None, bits, o,
                           workspace=torch.zeros(8, dtype=torch.uint8, device="cuda"))
