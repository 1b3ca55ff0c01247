"""GPU exact boxplus (Sec. II-B) against the oracle's FP64 exact boxplus.

The kernel evaluates the exact check function in FP32 on the hardware exp2
and log2, so it agrees with the FP64 oracle to rounding, not bit for bit.
Bounds used here: one check node within 4e-7 + 2^-22 |f| of the FP64 value
(two hardware log2 and exp2 results of about one ulp each, scaled by ln 2,
plus the final rounding); every message of the first three iterations
within TOL * max(|m64|, max |LLR| of the frame), TOL about eight times the
largest deviation seen; over whole decodes, the frames the oracle decodes
within the budget decided identically with equal iteration counts (frames
that never converge follow chaotic trajectories whose rounding-level
differences grow), frame error rates inside each other's binomial
intervals, and the exact decoder at least as good as min-sum on the same
frames."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 4e-6


@pytest.fixture(scope="module")
def pbp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1911_08868_amd as m
    return m


def _gpu(pbp, oc, llr, bp, pp=None, soft=True, dsnr=2.5):
    import torch
    code = pbp.Code(oc.N, oc.K, oc.crc_width, oc.crc_poly, dsnr)
    assert np.array_equal(code.info_idx, oc.info_idx)
    out = pbp.pp_mt_bp_decode(code, torch.from_numpy(llr).cuda(), bp, pp or pbp.PPParams(), soft=soft)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def test_single_check_node(orc, pbp):
    # N = 2, both bits information, one iteration: the u-side L of row 0 is
    # l0 boxplus l1; the values span the saturation range of the tanh form
    vals = np.array([0.0, 1e-3, 0.37, 1.0, 2.5, 7.0, 19.0, 38.0, 45.0, 90.0, 300.0], np.float32)
    a, b = np.meshgrid(np.concatenate([vals, -vals[1:]]), np.concatenate([vals, -vals[1:]]))
    llr = np.stack([a.ravel(), b.ravel()], 1).astype(np.float32)
    bp = pbp.BPParams(max_iter=1, stop=pbp.STOP_NONE, check=pbp.CHECK_EXACT)
    import torch
    code = pbp.Code(2, 2, 0, 0, 2.0)
    _, _, _, soft = pbp.pp_mt_bp_decode(code, torch.from_numpy(llr).cuda(), bp, pbp.PPParams(),
                                        soft=True)
    soft = soft.cpu().numpy()
    for f in range(llr.shape[0]):
        L, _ = orc.bp_run(llr[f], np.zeros(2, np.uint8), 1, fp32=False, exact=True)
        want = L[1, 0]
        assert abs(soft[f, 0] - want) <= 4e-7 + 2.0**-22 * abs(want), (llr[f], soft[f, 0], want)
        assert soft[f, 1] == llr[f, 1]          # f(prior 0, l0) = 0, plus l1
        if abs(want) > 1e-6:
            assert np.sign(soft[f, 0]) == np.sign(want)


@pytest.mark.parametrize("N,K,cw,poly,ppk,opk", [
    (64, 32, 8, 0x07, None, {}),
    (256, 144, 16, 0x1021, dict(mode=0, k=3, period_T=1, pool_Q=4, seed=2),
     dict(pp_mode=0, k=3, T=1, Q=4, seed=2)),
    (1024, 512, 16, 0x1021, dict(mode=0, k=4, period_T=2, pool_Q=8, seed=1),
     dict(pp_mode=0, k=4, T=2, Q=8, seed=1)),
    (128, 64, 8, 0x07, dict(mode=1, period_T=1, pool_Q=3, seed=5), dict(pp_mode=1, T=1, Q=3, seed=5)),
])
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_early_messages_within_rounding(orc, pbp, N, K, cw, poly, ppk, opk, iters):
    oc = orc.construct(N, K, 2.5, cw, poly)
    F = 48
    msg = synth.message_bits(N + iters, F, oc.K_msg)
    _, x = orc.encode(oc, msg)
    llr = synth.awgn_llr(x, 1.5, oc.K_msg, seed=N + iters)
    bp = pbp.BPParams(max_iter=iters, stop=pbp.STOP_NONE, check=pbp.CHECK_EXACT)
    pp = pbp.PPParams(**ppk) if ppk else None
    soft = _gpu(pbp, oc, llr, bp, pp)[3]
    ref = orc.decode(oc, llr, orc.DecodeParams(max_iter=iters, stop=orc.STOP_NONE, fp32=False,
                                               exact_boxplus=True, **opk), soft=True, threads=8)
    scale = np.maximum(np.abs(ref.soft_u), np.abs(llr).max(1, keepdims=True))
    ratio = np.abs(soft - ref.soft_u) / scale
    assert ratio.max() <= TOL, f"max relative deviation {ratio.max():.3e}"


def _frames(orc, N, K, cw, poly, F, snr, seed):
    oc = orc.construct(N, K, 2.5, cw, poly)
    msg = synth.message_bits(seed, F, oc.K_msg)
    _, x = orc.encode(oc, msg)
    return oc, msg, synth.awgn_llr(x, snr, oc.K_msg, seed=seed)


def _ci(k, n, z=2.576):
    """Wilson interval of a binomial proportion (99%)."""
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h


@pytest.mark.parametrize("N,K,cw,poly,snr,ppk,opk", [
    (256, 128, 16, 0x1021, 1.75, None, {}),
    (512, 256, 16, 0x1021, 1.75, dict(mode=0, k=4, period_T=10, pool_Q=8, seed=1),
     dict(pp_mode=0, k=4, T=10, Q=8, seed=1)),
])
def test_whole_decodes_agree(orc, pbp, N, K, cw, poly, snr, ppk, opk):
    F = 600
    oc, msg, llr = _frames(orc, N, K, cw, poly, F, snr, seed=N)
    bp = pbp.BPParams(max_iter=60, stop=pbp.STOP_CRC, check=pbp.CHECK_EXACT)
    pp = pbp.PPParams(**ppk) if ppk else None
    m, it, ok, _ = _gpu(pbp, oc, llr, bp, pp)
    ref = orc.decode(oc, llr, orc.DecodeParams(max_iter=60, stop=orc.STOP_CRC, fp32=False,
                                               exact_boxplus=True, **opk), threads=8)
    same = (m == ref.msg_hat).all(1) & (it == ref.iters) & (ok == ref.ok)
    stopped = ref.ok == 1
    assert stopped.sum() > F // 3
    assert same[stopped].mean() >= 0.98, f"only {same[stopped].mean():.3f} of converged frames agree"
    e_gpu, e_ref = int((m != msg).any(1).sum()), int((ref.msg_hat != msg).any(1).sum())
    lo, hi = _ci(e_ref, F)
    assert lo * F <= e_gpu <= hi * F, (e_gpu, e_ref)
    # exact BP is at least as good as min-sum on the same frames (up to noise)
    bp_ms = pbp.BPParams(max_iter=60, stop=pbp.STOP_CRC)
    m_ms = _gpu(pbp, oc, llr, bp_ms, pp, soft=False)[0]
    e_ms = int((m_ms != msg).any(1).sum())
    assert e_gpu <= e_ms + 3 * math.sqrt(max(e_ms, 1)), (e_gpu, e_ms)


@pytest.mark.parametrize("mode", [2, 3], ids=["current", "orig"])  # PP_ALG1, PP_ALG1_ORIG
@pytest.mark.parametrize("iters,first_reset", [(1, 0), (3, 1), (5, 2)])
def test_algorithm1_early_messages_within_rounding(orc, pbp, iters, first_reset, mode):
    # Algorithm 1 with the exact boxplus: its events depend on the draws only,
    # so both sides permute the same blocks; the u-side messages after a few
    # iterations (events after iterations 1 and 2 included) within rounding
    oc = orc.construct(256, 144, 2.5, 16, 0x1021)
    F = 48
    msg = synth.message_bits(300 + iters, F, oc.K_msg)
    _, x = orc.encode(oc, msg)
    llr = synth.awgn_llr(x, 1.5, oc.K_msg, seed=300 + iters)
    bp = pbp.BPParams(max_iter=iters, stop=pbp.STOP_NONE, check=pbp.CHECK_EXACT)
    t = dict(P_range=5, P_level=4, D=0, N_min=1, first_reset=first_reset, seed=4)
    soft = _gpu(pbp, oc, llr, bp, pbp.PPParams(mode=mode, **t))[3]
    ref = orc.decode(oc, llr, orc.DecodeParams(max_iter=iters, stop=orc.STOP_NONE, fp32=False,
                                               exact_boxplus=True, pp_mode=mode, **t),
                     soft=True, threads=8)
    scale = np.maximum(np.abs(ref.soft_u), np.abs(llr).max(1, keepdims=True))
    ratio = np.abs(soft - ref.soft_u) / scale
    assert ratio.max() <= TOL, f"max relative deviation {ratio.max():.3e}"


@pytest.mark.parametrize("mode", [2, 3], ids=["current", "orig"])  # PP_ALG1, PP_ALG1_ORIG
@pytest.mark.parametrize("N,K,table", [(512, 333, (9, 8, 50, 15)), (1024, 512, (2, 6, 8, 4))])
def test_algorithm1_whole_decodes_agree(orc, pbp, N, K, table, mode):
    # Table I parameter sets with the exact boxplus.  The events reset parts
    # of the graph every few iterations, which lets rounding-level differences
    # steer slowly converging frames apart (they stop at another iteration,
    # nearly always on the same message), so: frames the oracle decodes within
    # 20 iterations decided alike, 95% of all it decodes, and error counts
    # inside each other's intervals
    F = 300
    oc, msg, llr = _frames(orc, N, K, 24, 0x1864CFB, F, 2.25 if N == 1024 else 2.75, seed=N + 5)
    P_range, P_level, D, N_min = table
    t = dict(P_range=P_range, P_level=P_level, D=D, N_min=N_min, seed=6)
    bp = pbp.BPParams(max_iter=150, stop=pbp.STOP_CRC, it_min=3, check=pbp.CHECK_EXACT)
    m, it, ok, _ = _gpu(pbp, oc, llr, bp, pbp.PPParams(mode=mode, **t))
    ref = orc.decode(oc, llr, orc.DecodeParams(max_iter=150, stop=orc.STOP_CRC, it_min=3, fp32=False,
                                               exact_boxplus=True, pp_mode=mode, **t), threads=8)
    same = (m == ref.msg_hat).all(1) & (it == ref.iters) & (ok == ref.ok)
    stopped = ref.ok == 1
    early = stopped & (ref.iters <= 20)
    assert stopped.sum() > F // 3 and early.sum() > F // 4
    assert same[early].mean() >= 0.99, f"only {same[early].mean():.3f} of early frames agree"
    assert same[stopped].mean() >= 0.95, f"only {same[stopped].mean():.3f} of converged frames agree"
    e_gpu, e_ref = int((m != msg).any(1).sum()), int((ref.msg_hat != msg).any(1).sum())
    lo, hi = _ci(e_ref, F)
    assert lo * F <= e_gpu <= hi * F, (e_gpu, e_ref)


def test_large_workload_sampled(orc, pbp):
    # the 1024-bit code and last-4 schedule on 16384 frames; 40 sampled
    # frames and the slowest ones decoded by the oracle
    import torch
    F = 16384
    oc, msg, llr = _frames(orc, 1024, 512, 16, 0x1021, F, 2.0, seed=77)
    bp = pbp.BPParams(max_iter=100, stop=pbp.STOP_CRC, check=pbp.CHECK_EXACT)
    pp = pbp.PPParams(mode=0, k=4, period_T=10, pool_Q=8, seed=1)
    m, it, ok = _gpu(pbp, oc, llr, bp, pp, soft=False)
    rng = np.random.default_rng(1)
    pick = np.union1d(rng.choice(F, 40, replace=False), np.argsort(-it)[:8])
    ref = orc.decode(oc, llr[pick], orc.DecodeParams(max_iter=100, stop=orc.STOP_CRC, fp32=False,
                                                     exact_boxplus=True, pp_mode=0, k=4, T=10, Q=8,
                                                     seed=1), threads=8)
    same = (m[pick] == ref.msg_hat).all(1) & (it[pick] == ref.iters)
    stopped = ref.iters < 100
    assert same[stopped].mean() >= 0.95, f"only {same[stopped].mean():.3f} of sampled frames agree"
    assert int((m != msg).any(1).sum()) < F // 4


def test_exact_rejections(pbp):
    import torch
    code = pbp.Code(256, 144, 16, 0x1021, 2.5)
    llr = torch.zeros((4, 256), dtype=torch.float32, device="cuda")
    ex = dict(max_iter=5, stop=pbp.STOP_CRC, check=pbp.CHECK_EXACT)
    with pytest.raises(pbp.PolarError):      # exact takes no scale
        pbp.pp_mt_bp_decode(code, llr, pbp.BPParams(alpha=0.9375, **ex), pbp.PPParams())
    with pytest.raises(pbp.PolarError):      # no decision history with Algorithm 1 either
        pbp.pp_mt_bp_decode_trace(code, llr, pbp.BPParams(**ex),
                                  pbp.PPParams(mode=pbp.PP_ALG1, P_range=2, P_level=2, D=4, N_min=2), 8)
    with pytest.raises(pbp.PolarError):      # rho 3 is built for min-sum only
        pbp.pp_mt_bp_decode(code, llr, pbp.BPParams(**ex), pbp.PPParams(),
                            cfg=pbp.LaunchCfg(rho=3, slots=0, grid=0))
    with pytest.raises(pbp.PolarError):
        pbp.pp_mt_bp_decode_trace(code, llr, pbp.BPParams(**ex), None, 8)
    with pytest.raises(pbp.PolarError):      # unknown check function
        pbp.pp_mt_bp_decode(code, llr, pbp.BPParams(max_iter=5, check=7), pbp.PPParams())
