"""GPU parity of noise injection at the trellis events (the future-work
combination of Sec. V; noise-aided BP of Table I) against the FP32 oracle:
decided bits, iteration counts, verdicts and the u-side L messages
bit-exact (values equal, bits equal where nonzero), on the last-k and
full-permutation schedules, noise without permutation, Algorithm 1, the G
test and scaled min-sum; the 1024-bit workload on sampled frames; and the
argument checks."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pbp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1911_08868_amd as m
    return m


def _frames(orc, N, K, cw, poly, F, snr, seed):
    oc = orc.construct(N, K, 2.5, cw, poly)
    msg = synth.message_bits(seed, F, oc.K_msg)
    _, x = orc.encode(oc, msg)
    return oc, msg, synth.awgn_llr(x, snr, oc.K_msg, seed=seed)


def _gpu(pbp, oc, llr, bpk, ppk, soft=True):
    import torch
    code = pbp.Code(oc.N, oc.K, oc.crc_width, oc.crc_poly, 2.5)
    assert np.array_equal(code.info_idx, oc.info_idx)
    out = pbp.pp_mt_bp_decode(code, torch.from_numpy(llr).cuda(), pbp.BPParams(**bpk),
                              pbp.PPParams(**ppk), soft=soft)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _assert_same(got, ref, soft_ref=None, tag=""):
    m, it, ok = got[:3]
    bad = np.nonzero((m != ref.msg_hat).any(1) | (it != ref.iters) | (ok != ref.ok))[0]
    assert bad.size == 0, f"{tag}: frames {bad[:5]} differ, iters {it[bad[:5]]} vs {ref.iters[bad[:5]]}"
    if soft_ref is not None:
        a, b = got[3], soft_ref.astype(np.float32)
        assert np.array_equal(a, b), f"{tag}: soft messages differ"
        nz = a != 0
        assert np.array_equal(a.view(np.uint32)[nz], b.view(np.uint32)[nz]), f"{tag}: bits differ"


CASES = [
    # N, K, cw, poly, F, snr, bp kwargs, pp (GPU), oracle pp kwargs, sigma
    (256, 144, 16, 0x1021, 300, 2.0, dict(max_iter=60, stop=2),
     dict(mode=0, k=3, period_T=3, pool_Q=4, seed=5), dict(pp_mode=0, k=3, T=3, Q=4, seed=5), 0.6),
    (1024, 512, 16, 0x1021, 96, 1.75, dict(max_iter=80, stop=2, it_min=3),
     dict(mode=0, k=4, period_T=10, pool_Q=8, seed=1), dict(pp_mode=0, k=4, T=10, Q=8, seed=1), 0.6),
    (64, 40, 8, 0x07, 400, 1.5, dict(max_iter=33, stop=0),
     dict(mode=1, period_T=5, pool_Q=4, seed=9), dict(pp_mode=1, T=5, Q=4, seed=9), 0.3),
    (128, 64, 0, 0, 300, 2.0, dict(max_iter=40, stop=1),
     dict(mode=0, k=3, period_T=4, pool_Q=1, seed=2), dict(pp_mode=0, k=3, T=4, Q=1, seed=2), 0.6),
    (512, 256, 16, 0x1021, 160, 1.75, dict(max_iter=70, stop=2, alpha=0.9375),
     dict(mode=0, k=5, period_T=6, pool_Q=8, seed=4), dict(pp_mode=0, k=5, T=6, Q=8, seed=4), 0.45),
    # Algorithm 1: noise after each of its events (Table I parameter sets)
    (1024, 512, 24, 0x1864CFB, 64, 1.75, dict(max_iter=120, stop=2, it_min=3),
     dict(mode=2, P_range=2, P_level=6, D=8, N_min=4, seed=6),
     dict(pp_mode=2, P_range=2, P_level=6, D=8, N_min=4, seed=6), 0.6),
    (512, 333, 24, 0x1864CFB, 96, 2.5, dict(max_iter=150, stop=2, it_min=3),
     dict(mode=2, P_range=9, P_level=8, D=50, N_min=15, seed=7),
     dict(pp_mode=2, P_range=9, P_level=8, D=50, N_min=15, seed=7), 0.6),
    (64, 40, 8, 0x07, 300, 1.5, dict(max_iter=60, stop=2, alpha=0.9375),
     dict(mode=2, P_range=4, P_level=3, D=2, N_min=2, seed=8),
     dict(pp_mode=2, P_range=4, P_level=3, D=2, N_min=2, seed=8), 0.3),
]


@pytest.mark.parametrize("N,K,cw,poly,F,snr,bpk,ppk,opk,sigma", CASES)
def test_noise_injection_matches_oracle(orc, pbp, N, K, cw, poly, F, snr, bpk, ppk, opk, sigma):
    oc, msg, llr = _frames(orc, N, K, cw, poly, F, snr, seed=N + int(sigma * 10))
    got = _gpu(pbp, oc, llr, bpk, dict(noise_sigma=sigma, **ppk))
    ref = orc.decode(oc, llr, orc.DecodeParams(max_iter=bpk["max_iter"], stop=bpk["stop"],
                                               it_min=bpk.get("it_min", 1),
                                               alpha=bpk.get("alpha", 1.0), fp32=True,
                                               noise_sigma=float(np.float32(sigma)), **opk),
                     soft=True, threads=8)
    _assert_same(got, ref, ref.soft_u, f"N={N} sigma={sigma} {opk}")
    # the noise changed the decoding of some frame against the noiseless schedule
    plain = _gpu(pbp, oc, llr, bpk, ppk)
    assert not np.array_equal(plain[3], got[3])


def test_noise_on_the_large_workload_sampled(orc, pbp):
    F = 16384
    oc, msg, llr = _frames(orc, 1024, 512, 16, 0x1021, F, 2.0, seed=5)
    bpk = dict(max_iter=200, stop=2)
    ppk = dict(mode=0, k=4, period_T=10, pool_Q=8, seed=3)
    m, it, ok = _gpu(pbp, oc, llr, bpk, dict(noise_sigma=0.6, **ppk), soft=False)
    # frame indices enter the noise, so the oracle decodes a prefix of the
    # call (the first 1536 frames) and the sample is taken from it
    P = 1536
    rng = np.random.default_rng(2)
    pick = np.union1d(rng.choice(P, 40, replace=False), np.argsort(-it[:P])[:8])
    sel = llr[:P]
    ref = orc.decode(oc, sel, orc.DecodeParams(max_iter=200, stop=2, pp_mode=0, k=4, T=10, Q=8,
                                               seed=3, fp32=True, noise_sigma=0.6), threads=8)
    assert np.array_equal(m[pick], ref.msg_hat[pick])
    assert np.array_equal(it[pick], ref.iters[pick]) and np.array_equal(ok[pick], ref.ok[pick])


@pytest.mark.parametrize("mode", [2, 3], ids=["current", "orig"])  # PP_ALG1, PP_ALG1_ORIG
def test_algorithm1_noise_on_the_large_workload_sampled(orc, pbp, mode):
    # Algorithm 1 (Table I 200-iteration set) with noise at its events, 16384
    # frames of the 1024-bit code in one launch (two frames per CU, refills
    # from the queue); sampled frames of a prefix against the oracle
    F = 16384
    oc, msg, llr = _frames(orc, 1024, 512, 24, 0x1864CFB, F, 2.0, seed=8)
    bpk = dict(max_iter=200, stop=2, it_min=3)
    t = dict(P_range=2, P_level=6, D=8, N_min=4, seed=4)
    m, it, ok = _gpu(pbp, oc, llr, bpk, dict(mode=mode, noise_sigma=0.6, **t), soft=False)
    P = 1024
    rng = np.random.default_rng(4)
    pick = np.union1d(rng.choice(P, 40, replace=False), np.argsort(-it[:P])[:8])
    ref = orc.decode(oc, llr[:P], orc.DecodeParams(max_iter=200, stop=2, it_min=3, pp_mode=mode, fp32=True,
                                                   noise_sigma=0.6, **t), threads=8)
    assert np.array_equal(m[pick], ref.msg_hat[pick])
    assert np.array_equal(it[pick], ref.iters[pick]) and np.array_equal(ok[pick], ref.ok[pick])
    assert it[pick].max() > 60          # the sample holds long decodes (many events)


def test_noise_rejections(pbp):
    import torch
    code = pbp.Code(256, 144, 16, 0x1021, 2.5)
    llr = torch.zeros((4, 256), dtype=torch.float32, device="cuda")
    bp = pbp.BPParams(max_iter=5, stop=pbp.STOP_CRC)
    lastk = dict(mode=pbp.PP_LASTK, k=3, period_T=2, pool_Q=4, seed=1)
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(pbp.PolarError):
            pbp.pp_mt_bp_decode(code, llr, bp, pbp.PPParams(noise_sigma=bad, **lastk))
    with pytest.raises(pbp.PolarError):          # no events without a fixed schedule
        pbp.pp_mt_bp_decode(code, llr, bp, pbp.PPParams(noise_sigma=0.6))
    with pytest.raises(pbp.PolarError):          # Algorithm 1 with noise: min-sum only
        pbp.pp_mt_bp_decode(code, llr, pbp.BPParams(max_iter=5, check=pbp.CHECK_EXACT),
                            pbp.PPParams(mode=pbp.PP_ALG1, P_range=2, P_level=2, D=4, N_min=2,
                                         noise_sigma=0.6))
    with pytest.raises(pbp.PolarError):          # exact boxplus: min-sum only
        pbp.pp_mt_bp_decode(code, llr, pbp.BPParams(max_iter=5, check=pbp.CHECK_EXACT),
                            pbp.PPParams(noise_sigma=0.6, **lastk))
    with pytest.raises(pbp.PolarError):          # decision history: not with noise
        pbp.pp_mt_bp_decode_trace(code, llr, bp, pbp.PPParams(noise_sigma=0.6, **lastk), 8)
    with pytest.raises(pbp.PolarError):          # rho 3 is built without noise
        pbp.pp_mt_bp_decode(code, llr, bp, pbp.PPParams(noise_sigma=0.6, **lastk),
                            cfg=pbp.LaunchCfg(rho=3))
