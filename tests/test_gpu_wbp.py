"""GPU parity of weighted BP (forward and hand-written adjoint) against the
oracle: forward outputs bit-exact against the FP32 oracle; every weight
gradient entry (FP32 adjoint) against the oracle's FP64 adjoint of the same
FP32 forward, within that entry's own rounding bound; determinism across
runs; the autograd wrapper."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pbp():
    import torch
    assert torch.cuda.is_available()
    import paper_1911_08868_amd as m
    return m


def _setup(orc, N, K, F, seed, snr=1.5, cw=0, poly=0):
    oc = orc.construct(N, K, 2.5, cw, poly)
    msg = synth.message_bits(seed, F, oc.K_msg)
    u, x = orc.encode(oc, msg)
    return oc, u, synth.awgn_llr(x, snr, oc.K_msg, seed=seed)


def _gpu(pbp, oc, llr, w, T, pp, gout):
    import torch
    code = pbp.Code(oc.N, oc.K, oc.crc_width, oc.crc_poly, 2.5)
    assert np.array_equal(code.info_idx, oc.info_idx)
    d_llr = torch.from_numpy(llr).cuda()
    d_w = torch.from_numpy(w.astype(np.float32)).cuda()
    F = llr.shape[0]
    ws = torch.empty(max(pbp.wbp_workspace_bytes(code, F, T), 1), dtype=torch.uint8, device="cuda")
    out = torch.empty((F, oc.N), dtype=torch.float32, device="cuda")
    pbp.wbp_forward(code, d_llr, d_w, pp, out, ws)
    gw = torch.empty_like(d_w)
    pbp.wbp_backward(code, d_llr, d_w, pp, torch.from_numpy(gout.astype(np.float32)).cuda(), gw, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy(), gw.cpu().numpy()


U32 = 2.0 ** -24


def _check_grad(gw, ref, absum, F, extra_abs=0.0):
    """Element-wise bound on an FP32 adjoint.  The forward messages are
    bit-exact, so the GPU routes every min-sum derivative as the oracle does,
    and the two adjoints differ by rounding only.  Each weight entry of
    iteration t is a sum over paths of products of local derivatives; a path
    crosses at most 2 n (T - t) stage steps, and the GPU rounds at most 5
    times per step (the weight product, the sum inside the processing element,
    the accumulator, and a group boundary's sum), then once for the product
    with the forward message and at most F - 1 times summing frames.  With k
    roundings on every path the error is at most k u / (1 - k u) times the
    sum of the paths' magnitudes (absum, from the oracle's magnitude pass),
    u = 2^-24; the oracle's own FP64 rounding adds far less than 1e-12 of it.
    extra_abs: a further absolute allowance per entry (an FP32 loss gradient
    that enters the adjoint already rounded)."""
    T, n = ref.shape[0], ref.shape[1]
    t = np.arange(T).reshape(T, 1, 1, 1)
    k = 10 * n * (T - t) + F + 1
    gamma = k * U32 / (1 - k * U32)
    bound = (gamma + 1e-12) * absum + extra_abs + 1e-30
    err = np.abs(gw.astype(np.float64) - ref)
    bad = err > bound
    assert not bad.any(), (f"{int(bad.sum())} of {bad.size} gradient entries outside their bound; "
                           f"worst err/bound {float((err / bound).max()):.3g}")
    return bound


@pytest.mark.parametrize("N,K,T,F,pp", [(16, 8, 2, 7, None), (16, 8, 3, 64, (2, 1, 2)),
                                        (32, 16, 4, 33, (3, 2, 3)), (256, 144, 10, 96, None),
                                        (256, 144, 10, 50, (4, 3, 8)), (64, 32, 5, 130, None),
                                        (1024, 512, 3, 9, (5, 1, 8))])
def test_weighted_forward_and_adjoint(orc, pbp, N, K, T, F, pp):
    n = N.bit_length() - 1
    oc, u, llr = _setup(orc, N, K, F, seed=N + T + F)
    rng = np.random.default_rng(N * T)
    w = rng.uniform(0.7, 1.3, (T, n, 2, N)).astype(np.float32).astype(np.float64)
    gout = rng.normal(size=(F, N)).astype(np.float32).astype(np.float64)
    gout[:, oc.frozen.astype(bool)] = 0.0
    if pp:
        k, tev, Q = pp
        opp = orc.WbpParams(pp_mode=orc.PP_LASTK, k=k, T_ev=tev, Q=Q, seed=7, fp32=True)
        gpp = pbp.PPParams(mode=pbp.PP_LASTK, k=k, period_T=tev, pool_Q=Q, seed=7)
    else:
        opp = orc.WbpParams(fp32=True)
        gpp = None
    out, gw = _gpu(pbp, oc, llr, w, T, gpp, gout)
    ref_out = orc.wbp_forward(oc, llr, w, opp)
    assert np.array_equal(out.view(np.uint32), ref_out.astype(np.float32).view(np.uint32))
    ref_gw, _, absum = orc.wbp_backward(oc, llr, w, opp, gout, want_abs=True)
    bound = _check_grad(gw, ref_gw, absum, F)
    # the last R sweep never reaches the output
    assert np.all(gw[T - 1, :, 1] == 0.0)
    # entries the oracle gives exactly zero (no path) are exactly zero here
    assert np.all(gw[absum == 0] == 0.0)
    # the bound checks almost every entry of the later iterations, whose
    # paths do not cancel; an entry with bound >= |g| is the small remainder
    # of path sums far larger than itself (condition number above 1 / (k u)),
    # which no FP32 evaluation order resolves
    nz = ref_gw != 0
    late = nz & (np.arange(T).reshape(T, 1, 1, 1) >= T // 2)
    assert (bound[late] < 0.1 * np.abs(ref_gw[late])).mean() > 0.95


def test_weighted_gradient_is_deterministic(orc, pbp):
    oc, u, llr = _setup(orc, 256, 144, 300, seed=5)
    rng = np.random.default_rng(1)
    w = rng.uniform(0.8, 1.2, (6, 8, 2, 256))
    g = rng.normal(size=(300, 256))
    a = _gpu(pbp, oc, llr, w, 6, None, g)[1]
    b = _gpu(pbp, oc, llr, w, 6, None, g)[1]
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_unit_weights_reproduce_decoder_soft_output(orc, pbp):
    import torch
    oc, u, llr = _setup(orc, 256, 144, 40, seed=9, snr=2.0, cw=16, poly=0x1021)
    code = pbp.Code(256, 144, 16, 0x1021, 2.5)
    T = 7
    dec = pbp.wbp.WeightedBPDecoder(code, T)
    out = dec(torch.from_numpy(llr).cuda()).detach().cpu().numpy()
    msg, iters, ok, soft = pbp.bp_decode(code, torch.from_numpy(llr).cuda(),
                                         pbp.BPParams(max_iter=T, stop=pbp.STOP_NONE), soft=True)
    info = oc.info_idx
    # equal values; the decoder's check function may give the other sign of zero
    s = soft.cpu().numpy()[:, info]
    o = out[:, info]
    assert np.array_equal(o, s)
    assert np.array_equal(o.view(np.uint32)[o != 0], s.view(np.uint32)[o != 0])


def test_autograd_training_step(orc, pbp):
    import torch
    oc, u, llr = _setup(orc, 64, 32, 256, seed=11, snr=2.0)
    code = pbp.Code(64, 32, 0, 0, 2.5)
    dec = pbp.wbp.WeightedBPDecoder(code, 4)
    x = torch.from_numpy(llr).cuda()
    info = torch.from_numpy(oc.info_idx.astype(np.int64)).cuda()
    ub = torch.from_numpy(u[:, oc.info_idx]).cuda()
    loss = pbp.wbp.bce_on_information_bits(dec(x), ub, info)
    loss.backward()
    g = dec.weight.grad.detach().cpu().numpy().astype(np.float64)
    # d loss / d o from the same BCE, then the oracle's adjoint
    o = torch.from_numpy(orc.wbp_forward(oc, llr, np.ones((4, 6, 2, 64)), orc.WbpParams(fp32=True)))
    o.requires_grad_(True)
    lo = o[:, torch.from_numpy(oc.info_idx.astype(np.int64))]
    uu = torch.from_numpy(u[:, oc.info_idx]).double()
    l2 = (uu * torch.nn.functional.softplus(lo) + (1 - uu) * torch.nn.functional.softplus(-lo)).mean()
    l2.backward()
    ref, _, absum = orc.wbp_backward(oc, llr, np.ones((4, 6, 2, 64)), orc.WbpParams(fp32=True),
                                     o.grad.numpy(), want_abs=True)
    # the loss gradient enters from torch's FP32 kernels: per output row
    # (sigmoid(o) - target) / count with an absolute error below 4 u / count
    # (the difference of two numbers of magnitude at most 1), carried to each
    # weight entry through the magnitudes of its paths from the rows
    unit = np.zeros((256, 64))
    unit[:, oc.info_idx] = 1.0 / (256 * oc.K)
    _, _, abs_unit = orc.wbp_backward(oc, llr, np.ones((4, 6, 2, 64)), orc.WbpParams(fp32=True),
                                      unit, want_abs=True)
    k = 10 * 6 * 4 + 256 + 1
    _check_grad(g, ref, absum, 256, extra_abs=4 * U32 * (1 + k * U32 * 2) * abs_unit)
    assert abs(loss.item() - l2.item()) < 1e-5 * max(1.0, abs(l2.item()))


@pytest.mark.parametrize("N,K,T,F,pp", [(2048, 1024, 3, 5, None), (2048, 1100, 4, 3, (5, 1, 4)),
                                        (4096, 2048, 3, 3, (5, 1, 8)), (4096, 2072, 2, 3, None)])
def test_weighted_large_frames(orc, pbp, N, K, T, F, pp):
    # N >= 2048: one frame per workgroup, the adjoint streams its arrays
    # through a per-workgroup scratch
    n = N.bit_length() - 1
    oc, u, llr = _setup(orc, N, K, F, seed=N + T)
    rng = np.random.default_rng(T)
    w = rng.uniform(0.7, 1.3, (T, n, 2, N)).astype(np.float32).astype(np.float64)
    gout = rng.normal(size=(F, N)).astype(np.float32).astype(np.float64)
    gout[:, oc.frozen.astype(bool)] = 0.0
    if pp:
        k, tev, Q = pp
        opp = orc.WbpParams(pp_mode=orc.PP_LASTK, k=k, T_ev=tev, Q=Q, seed=3, fp32=True)
        gpp = pbp.PPParams(mode=pbp.PP_LASTK, k=k, period_T=tev, pool_Q=Q, seed=3)
    else:
        opp, gpp = orc.WbpParams(fp32=True), None
    out, gw = _gpu(pbp, oc, llr, w, T, gpp, gout)
    assert np.array_equal(out.view(np.uint32), orc.wbp_forward(oc, llr, w, opp).astype(np.float32).view(np.uint32))
    ref_gw, _, absum = orc.wbp_backward(oc, llr, w, opp, gout, want_abs=True)
    _check_grad(gw, ref_gw, absum, F)
    assert np.all(gw[T - 1, :, 1] == 0.0)


@pytest.mark.parametrize("N,K,T,F,pp", [(4096, 2048, 2, 260, None), (2048, 1100, 3, 515, (5, 1, 4))])
def test_weighted_large_frames_more_than_the_grid(orc, pbp, N, K, T, F, pp):
    # more frames than the fixed grid (256 workgroups at N = 4096, 512 at
    # N = 2048): the first workgroups take a second frame and add into their
    # partial; with the permuted range, the trellis changes at every iteration
    n = N.bit_length() - 1
    oc, u, llr = _setup(orc, N, K, F, seed=12 + N)
    rng = np.random.default_rng(12)
    w = rng.uniform(0.8, 1.2, (T, n, 2, N)).astype(np.float32).astype(np.float64)
    gout = rng.normal(size=(F, N)).astype(np.float32).astype(np.float64)
    if pp:
        k, tev, Q = pp
        opp = orc.WbpParams(pp_mode=orc.PP_LASTK, k=k, T_ev=tev, Q=Q, seed=5, fp32=True)
        gpp = pbp.PPParams(mode=pbp.PP_LASTK, k=k, period_T=tev, pool_Q=Q, seed=5)
    else:
        opp, gpp = orc.WbpParams(fp32=True), None
    out, gw = _gpu(pbp, oc, llr, w, T, gpp, gout)
    assert np.array_equal(out.view(np.uint32), orc.wbp_forward(oc, llr, w, opp).astype(np.float32).view(np.uint32))
    ref_gw, _, absum = orc.wbp_backward(oc, llr, w, opp, gout, want_abs=True)
    _check_grad(gw, ref_gw, absum, F)
    again = _gpu(pbp, oc, llr, w, T, gpp, gout)[1]
    assert np.array_equal(gw.view(np.uint32), again.view(np.uint32))


@pytest.mark.parametrize("N,K,T,F,pp", [(64, 32, 3, 32 * 300 + 5, None), (16, 8, 2, 128 * 270 + 3, None),
                                        (256, 144, 3, 8 * 300 + 3, None), (1024, 512, 2, 600, None),
                                        (256, 144, 4, 8 * 300 + 5, (4, 1, 8)), (1024, 512, 3, 520, (5, 2, 4))])
def test_weighted_gradient_over_many_workgroups(orc, pbp, N, K, T, F, pp):
    # more batches of frames than the adjoint's fixed grid (256 workgroups up
    # to N = 256, 512 above): the first workgroups take a second batch and add
    # into their partial, the last batch is ragged, and more than 64 partials
    # take both levels of the gradient reduction; with the permuted range the
    # one-wave adjoint takes its other flush (the partial loaded at the flush)
    n = N.bit_length() - 1
    oc, u, llr = _setup(orc, N, K, F, seed=3 + F)
    rng = np.random.default_rng(F)
    w = rng.uniform(0.7, 1.3, (T, n, 2, N)).astype(np.float32).astype(np.float64)
    gout = rng.normal(size=(F, N)).astype(np.float32).astype(np.float64)
    if pp:
        k, tev, Q = pp
        opp = orc.WbpParams(pp_mode=orc.PP_LASTK, k=k, T_ev=tev, Q=Q, seed=9, fp32=True)
        gpp = pbp.PPParams(mode=pbp.PP_LASTK, k=k, period_T=tev, pool_Q=Q, seed=9)
    else:
        opp, gpp = orc.WbpParams(fp32=True), None
    out, gw = _gpu(pbp, oc, llr, w, T, gpp, gout)
    assert np.array_equal(out.view(np.uint32), orc.wbp_forward(oc, llr, w, opp).astype(np.float32).view(np.uint32))
    ref_gw, _, absum = orc.wbp_backward(oc, llr, w, opp, gout, want_abs=True)
    _check_grad(gw, ref_gw, absum, F)


def test_weighted_empty_batch_gives_zero_gradient(pbp):
    import torch
    code = pbp.Code(64, 32, 0, 0, 2.5)
    w = torch.ones((3, 6, 2, 64), dtype=torch.float32, device="cuda")
    gw = torch.full_like(w, 5.0)
    llr = torch.empty((0, 64), dtype=torch.float32, device="cuda")
    ws = torch.empty(1, dtype=torch.uint8, device="cuda")
    pbp.wbp_backward(code, llr, w, None, torch.empty((0, 64), dtype=torch.float32, device="cuda"), gw, ws)
    torch.cuda.synchronize()
    assert torch.count_nonzero(gw).item() == 0


def test_weighted_forward_without_checkpoints(orc, pbp):
    import torch
    oc, u, llr = _setup(orc, 256, 144, 70, seed=21)
    code = pbp.Code(256, 144, 0, 0, 2.5)
    rng = np.random.default_rng(2)
    w = torch.from_numpy(rng.uniform(0.8, 1.2, (5, 8, 2, 256)).astype(np.float32)).cuda()
    x = torch.from_numpy(llr).cuda()
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=3, period_T=2, pool_Q=4, seed=3)
    a = torch.empty((70, 256), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ws = torch.empty(pbp.wbp_workspace_bytes(code, 70, 5), dtype=torch.uint8, device="cuda")
    pbp.wbp_forward(code, x, w, pp, a, ws)
    pbp.wbp_forward(code, x, w, pp, b, None)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    dec = pbp.wbp.WeightedBPDecoder(code, 5)
    with torch.no_grad():
        o = dec(x)
    ref = orc.wbp_forward(oc, llr, np.ones((5, 8, 2, 256)), orc.WbpParams(fp32=True))
    assert np.array_equal(o.cpu().numpy().view(np.uint32), ref.astype(np.float32).view(np.uint32))


def test_two_forwards_before_backward(orc, pbp):
    # each forward call keeps its own checkpoints
    import torch
    oc, u, llr1 = _setup(orc, 64, 32, 40, seed=31)
    _, _, llr2 = _setup(orc, 64, 32, 40, seed=32)
    code = pbp.Code(64, 32, 0, 0, 2.5)
    dec = pbp.wbp.WeightedBPDecoder(code, 3)
    g = torch.from_numpy(np.random.default_rng(4).normal(size=(40, 64)).astype(np.float32)).cuda()
    o1 = dec(torch.from_numpy(llr1).cuda())
    o2 = dec(torch.from_numpy(llr2).cuda())
    (o1 * g).sum().backward()
    g1 = dec.weight.grad.clone()
    dec.weight.grad = None
    (o2 * g).sum().backward()
    ref1, _, absum = orc.wbp_backward(oc, llr1, np.ones((3, 6, 2, 64)), orc.WbpParams(fp32=True),
                                      g.cpu().numpy().astype(np.float64), want_abs=True)
    _check_grad(g1.cpu().numpy(), ref1, absum, 40)
