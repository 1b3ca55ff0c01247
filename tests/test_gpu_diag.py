"""GPU parity of the error-class diagnostics (Sec. II-C) against the oracle:
the decision-hash history bit-exact (every column of every frame), decoded
bits, iteration counts and verdicts bit-exact, and the error classes and
decision periods exact, on plain BP, the fixed last-k and full-permutation
schedules, the G test, scaled min-sum and Algorithm 1; at the 1024-bit
workload on sampled frames; and the classifier on hand-built histories."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "published_constants.json")))
TABLE1 = GOLD["table1_pp_bp_parameters"]


@pytest.fixture(scope="module")
def pbp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1911_08868_amd as m
    return m


def _frames(orc, N, K, cw, poly, F, snr, seed, dsnr=2.5):
    oc = orc.construct(N, K, dsnr, cw, poly)
    msg = synth.message_bits(seed, F, oc.K_msg)
    _, x = orc.encode(oc, msg)
    return oc, msg, synth.awgn_llr(x, snr, oc.K_msg, seed=seed)


def _gpu_trace(pbp, oc, llr, H, bp_kw, pp_kw, dsnr=2.5):
    import torch
    code = pbp.Code(oc.N, oc.K, oc.crc_width, oc.crc_poly, dsnr)
    assert np.array_equal(code.info_idx, oc.info_idx)
    bp = pbp.BPParams(**bp_kw)
    pp = pbp.PPParams(**pp_kw) if pp_kw else None
    out = pbp.pp_mt_bp_decode_trace(code, torch.from_numpy(llr).cuda(), bp, pp, H)
    torch.cuda.synchronize()
    return code, bp, pp, out


def _gpu_classes(pbp, out, msg):
    import torch
    m, it, ok, hist = out
    cls, per = pbp.classify_errors(m, torch.from_numpy(msg).cuda(), ok, it, hist)
    torch.cuda.synchronize()
    return cls.cpu().numpy(), per.cpu().numpy()


def _host(out):
    m, it, ok, hist = out
    return m.cpu().numpy(), it.cpu().numpy(), ok.cpu().numpy(), hist.cpu().numpy().view(np.uint64)


CASES = [
    # N, K, cw, poly, F, snr, H, bp kwargs, pp kwargs (GPU), oracle pp kwargs
    (256, 128, 16, 0x1021, 300, 1.5, 16, dict(max_iter=60, stop=2), None, {}),
    (1024, 512, 16, 0x1021, 96, 1.75, 32,
     dict(max_iter=80, stop=2, it_min=3), dict(mode=0, k=4, period_T=10, pool_Q=8, seed=7),
     dict(pp_mode=0, k=4, T=10, Q=8, seed=7)),
    (64, 40, 8, 0x07, 400, 1.0, 5, dict(max_iter=41, stop=0),
     dict(mode=1, period_T=6, pool_Q=4, seed=3), dict(pp_mode=1, T=6, Q=4, seed=3)),
    (128, 64, 0, 0, 300, 1.5, 12, dict(max_iter=50, stop=1), None, {}),
    (512, 256, 16, 0x1021, 160, 1.5, 64, dict(max_iter=90, stop=2, alpha=0.9375),
     dict(mode=0, k=5, period_T=7, pool_Q=8, seed=11), dict(pp_mode=0, k=5, T=7, Q=8, seed=11)),
]


@pytest.mark.parametrize("N,K,cw,poly,F,snr,H,bpk,ppk,opk", CASES)
def test_history_and_classes_match_oracle(orc, pbp, N, K, cw, poly, F, snr, H, bpk, ppk, opk):
    oc, msg, llr = _frames(orc, N, K, cw, poly, F, snr, seed=N + H)
    _, _, _, out = _gpu_trace(pbp, oc, llr, H, bpk, ppk)
    m, it, ok, hist = _host(out)
    p = orc.DecodeParams(max_iter=bpk["max_iter"], stop=bpk["stop"], it_min=bpk.get("it_min", 1),
                         alpha=bpk.get("alpha", 1.0), fp32=True, **opk)
    ref, rhist = orc.decode_trace(oc, llr, p, H, threads=8)
    tag = f"N={N} H={H} {opk}"
    bad = np.nonzero((m != ref.msg_hat).any(1) | (it != ref.iters) | (ok != ref.ok))[0]
    assert bad.size == 0, f"{tag}: frames {bad[:5]} differ"
    bad = np.nonzero((hist != rhist).any(1))[0]
    assert bad.size == 0, f"{tag}: histories of frames {bad[:5]} differ"
    cls, per = _gpu_classes(pbp, out, msg)
    rcls, rper = orc.classify(ref.msg_hat, msg, ref.ok, ref.iters, rhist)
    assert np.array_equal(cls, rcls) and np.array_equal(per, rper), tag
    wrong = (m != msg).any(1)
    assert wrong.sum() > 0, f"{tag}: the case should contain failed frames"


@pytest.mark.parametrize("mode", [2, 3], ids=["current", "orig"])  # PP_ALG1, PP_ALG1_ORIG
def test_algorithm1_history_matches_oracle(orc, pbp, mode):
    t = TABLE1["N512_Nitmax20000"]
    oc, msg, llr = _frames(orc, 512, 333, 24, 0x1864CFB, 48, 2.0, seed=31)
    ppk = dict(mode=mode, P_range=t["P_range"], P_level=t["P_level"], D=t["D"], N_min=t["N_min"], seed=5)
    _, _, _, out = _gpu_trace(pbp, oc, llr, 24, dict(max_iter=120, stop=2, it_min=3), ppk)
    m, it, ok, hist = _host(out)
    p = orc.DecodeParams(max_iter=120, stop=2, it_min=3, pp_mode=mode, P_range=t["P_range"],
                         P_level=t["P_level"], D=t["D"], N_min=t["N_min"], seed=5, fp32=True)
    ref, rhist = orc.decode_trace(oc, llr, p, 24, threads=8)
    assert np.array_equal(m, ref.msg_hat) and np.array_equal(it, ref.iters)
    assert np.array_equal(ok, ref.ok)
    assert np.array_equal(hist, rhist)
    cls, per = _gpu_classes(pbp, out, msg)
    rcls, rper = orc.classify(ref.msg_hat, msg, ref.ok, ref.iters, rhist)
    assert np.array_equal(cls, rcls) and np.array_equal(per, rper)


def test_trace_decodes_like_the_plain_kernel(orc, pbp):
    # the 1024-bit headline code and schedule on 8192 frames: the trace kernel
    # decides exactly as the kernel without history
    import torch
    oc, msg, llr = _frames(orc, 1024, 512, 16, 0x1021, 8192, 1.75, seed=41)
    bpk = dict(max_iter=200, stop=2)
    ppk = dict(mode=0, k=4, period_T=10, pool_Q=8, seed=1)
    code, bp, pp, out = _gpu_trace(pbp, oc, llr, 32, bpk, ppk)
    m0, it0, ok0 = pbp.pp_mt_bp_decode(code, torch.from_numpy(llr).cuda(), bp, pp)
    torch.cuda.synchronize()
    m, it, ok, hist = _host(out)
    assert np.array_equal(m, m0.cpu().numpy()) and np.array_equal(it, it0.cpu().numpy())
    assert np.array_equal(ok, ok0.cpu().numpy())
    # sampled frames against the oracle, one by one
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(8192, 40, replace=False))
    pick = np.union1d(pick, np.argsort(-it)[:8])          # and the longest decodes
    p = orc.DecodeParams(max_iter=200, stop=2, pp_mode=0, k=4, T=10, Q=8, seed=1, fp32=True)
    ref, rhist = orc.decode_trace(oc, llr[pick], p, 32, threads=8)
    assert np.array_equal(it[pick], ref.iters)
    assert np.array_equal(hist[pick], rhist)
    cls, per = _gpu_classes(pbp, out, msg)
    rcls, rper = orc.classify(ref.msg_hat, msg[pick], ref.ok, ref.iters, rhist)
    assert np.array_equal(cls[pick], rcls) and np.array_equal(per[pick], rper)


def test_classifier_on_hand_built_histories(orc, pbp):
    # random histories with planted periods, ring rotations and iteration
    # counts below and above H, on many frames (several per workgroup)
    import torch
    rng = np.random.default_rng(3)
    F, H, K = 1000, 16, 37
    iters = rng.integers(1, 60, F).astype(np.int32)
    hist = rng.integers(0, 2**63, (F, H), dtype=np.int64).view(np.uint64)
    for f in range(F):
        p = int(rng.integers(0, 6))
        if p:
            W = min(H, int(iters[f]))
            base = rng.integers(0, 4, p).astype(np.uint64)
            for i in range(W):
                hist[f, (iters[f] - W + i) % H] = base[i % p]
    msg = rng.integers(0, 2, (F, K)).astype(np.uint8)
    hat = msg.copy()
    flip = rng.random(F) < 0.8
    hat[flip, rng.integers(0, K, flip.sum())] ^= 1
    ok = (rng.random(F) < 0.2).astype(np.uint8)
    rcls, rper = orc.classify(hat, msg, ok, iters, hist)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cls, per = pbp.classify_errors(dev(hat), dev(msg), dev(ok), dev(iters), dev(hist.view(np.int64)))
    torch.cuda.synchronize()
    assert np.array_equal(cls.cpu().numpy(), rcls)
    assert np.array_equal(per.cpu().numpy(), rper)
    assert set(rcls.tolist()) == {0, 1, 2, 3}


def test_trace_rejects_bad_history_length(pbp):
    import torch
    code = pbp.Code(64, 32, 8, 0x07, 2.0)
    llr = torch.zeros((4, 64), dtype=torch.float32, device="cuda")
    for H in (0, 65):
        with pytest.raises((pbp.PolarError, RuntimeError)):
            pbp.pp_mt_bp_decode_trace(code, llr, pbp.BPParams(max_iter=5, stop=2), None, H)


def test_trace_and_classify_edge_cases(orc, pbp):
    # empty batch, one iteration, a ring longer than the decode, and the
    # classifier's argument checks
    import torch
    code = pbp.Code(64, 40, 8, 0x07, 2.5)
    empty = torch.zeros((0, 64), dtype=torch.float32, device="cuda")
    m, it, ok, hist = pbp.pp_mt_bp_decode_trace(code, empty, pbp.BPParams(max_iter=5, stop=2), None, 4)
    assert m.shape == (0, code.K_msg) and hist.shape == (0, 4)
    cls, per = pbp.classify_errors(m, m.clone(), ok, it, hist)
    assert cls.numel() == 0
    oc, msg, llr = _frames(orc, 64, 40, 8, 0x07, 50, 1.0, seed=3)
    _, _, _, out = _gpu_trace(pbp, oc, llr, 64, dict(max_iter=1, stop=0), None)
    m, it, ok, hist = _host(out)
    assert np.all(it == 1) and np.all(hist[:, 1:] == 0)
    ref, rhist = orc.decode_trace(oc, llr, orc.DecodeParams(max_iter=1, stop=0, fp32=True), 64)
    assert np.array_equal(hist, rhist)
    cls, per = _gpu_classes(pbp, out, msg)
    assert np.all(per == 0)                  # one sample shows no period
    with pytest.raises(pbp.PolarError):      # ring length beyond 64
        pbp.classify_errors(out[0], torch.from_numpy(msg).cuda(), out[2], out[1],
                            torch.zeros((50, 65), dtype=torch.int64, device="cuda"))
