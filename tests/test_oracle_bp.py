"""Pins for the oracle's BP core (Sec. II-B): the processing element and check
function on cases with closed forms, MAP on the cycle-free N = 2 graph,
noiseless decoding, codeword symmetry, relabelling of permuted graphs, and
FP32 against FP64."""
import itertools
import math

import numpy as np
import pytest

import synth


def _map_llrs_n2(l0, l1, frozen0):
    """Exact a-posteriori LLRs of u0, u1 for x = (u0^u1, u1) by enumeration."""
    def lik(x, l):  # p(y|x) up to a common factor, from the channel LLR
        return math.exp(l / 2) if x == 0 else math.exp(-l / 2)
    post = {}
    for u0, u1 in itertools.product([0, 1], repeat=2):
        if frozen0 and u0 == 1:
            continue
        post[(u0, u1)] = lik(u0 ^ u1, l0) * lik(u1, l1)
    p = lambda i, b: sum(v for k, v in post.items() if k[i] == b)
    out = []
    for i in range(2):
        if frozen0 and i == 0:
            out.append(math.inf)
        else:
            out.append(math.log(p(i, 0) / p(i, 1)))
    return out


@pytest.mark.parametrize("l0,l1", [(1.3, -0.4), (-2.0, 3.5), (0.2, 0.1), (-1.1, -0.7)])
@pytest.mark.parametrize("frozen0", [False, True])
def test_exact_boxplus_is_map_on_n2(orc, l0, l1, frozen0):
    fr = np.array([1 if frozen0 else 0, 0], np.uint8)
    L, R = orc.bp_run(np.array([l0, l1], np.float32), fr, 1, fp32=False, exact=True)
    post = L[1] + R[1]
    want = _map_llrs_n2(float(np.float32(l0)), float(np.float32(l1)), frozen0)
    if not frozen0:
        assert post[0] == pytest.approx(want[0], rel=1e-12)
    assert post[1] == pytest.approx(want[1], rel=1e-12)


def test_minsum_pe_closed_form(orc):
    # N = 2, both bits information: L(u0) = a sgn sgn min, L(u1) = a*f(0, l0) + l1
    for l0, l1, a in [(1.5, -0.25, 1.0), (-3.0, -2.0, 0.9375), (0.5, 4.0, 0.9375)]:
        L, R = orc.bp_run(np.array([l0, l1], np.float32), np.zeros(2, np.uint8), 1, alpha=a)
        want0 = np.float32(a) * np.float32(min(abs(l0), abs(l1))) * np.sign(l0) * np.sign(l1)
        assert L[1, 0] == np.float32(want0)
        assert L[1, 1] == np.float32(l1)           # f(R=0, l0) = +-0, plus l1
        # channel-side R messages after the R sweep: both carry f(0, .) = +-0
        assert R[0, 0] == 0.0 and R[0, 1] == 0.0
    # frozen u0: prior +inf passes the other argument through unchanged
    L, R = orc.bp_run(np.array([-0.75, 2.0], np.float32), np.array([1, 0], np.uint8), 1)
    assert L[1, 1] == np.float32(-0.75 + 2.0)
    assert R[0, 0] == np.float32(2.0)              # f(inf, l1 + 0) = l1
    assert R[0, 1] == np.float32(-0.75)            # f(inf, l0) + R(u1) = l0 + 0


def test_signed_zero_rules(orc):
    # f(+0, y) carries the xor of the sign bits: -0 when y < 0
    L, R = orc.bp_run(np.array([0.0, -2.0], np.float32), np.zeros(2, np.uint8), 1)
    assert L[1, 0] == 0.0 and math.copysign(1.0, L[1, 0]) == -1.0
    # decision ties (R + L = +-0) decide 0
    res = orc.decode(orc.Code(2, 2, np.array([0, 1], np.int32), np.zeros(2, np.uint8)),
                     np.array([[0.0, -2.0]], np.float32),
                     orc.DecodeParams(max_iter=1, stop=orc.STOP_NONE))
    assert res.msg_hat[0, 0] == 0


@pytest.mark.parametrize("N,K", [(64, 32), (256, 128), (1024, 512)])
def test_noiseless_decodes_in_one_iteration(orc, N, K):
    code = orc.construct(N, K, 2.0)
    msg = synth.message_bits(10, 20, K)
    u, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 3.0, K, seed=1, noiseless=True)
    res = orc.decode(code, llr, orc.DecodeParams(max_iter=5, stop=orc.STOP_G, it_min=1))
    assert np.all(res.iters == 1)
    assert np.array_equal(res.msg_hat, msg)


@pytest.mark.parametrize("fp32", [True, False])
def test_codeword_symmetry(orc, fp32):
    # BP state for codeword x equals the all-zero state with signs flipped by the
    # partial codewords, so u_hat(x) = u_hat(0) xor u exactly
    code = orc.construct(256, 128, 2.5, 16, 0x1021)
    msg = synth.message_bits(3, 40, code.K_msg)
    u, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 2.0, code.K_msg, seed=9)
    llr0 = llr * (1 - 2 * x.astype(np.float32))     # same noise on the all-zero word
    sign = 1 - 2 * u.astype(np.float64)
    for it in (1, 5, 30):
        p = orc.DecodeParams(max_iter=it, stop=orc.STOP_NONE, fp32=fp32)
        r = orc.decode(code, llr, p, soft=True)
        r0 = orc.decode(code, llr0, p, soft=True)
        np.testing.assert_array_equal(np.abs(r.soft_u), np.abs(r0.soft_u))
        nz = r0.soft_u != 0
        np.testing.assert_array_equal((r.soft_u * sign)[nz], r0.soft_u[nz])
        # decisions follow u_hat(x) = u_hat(0) xor u except on exact ties (soft = +-0),
        # which decide 0 on both sides
        tie = ~nz[:, code.info_idx[:code.K_msg]]
        assert np.array_equal((r.msg_hat != (r0.msg_hat ^ msg)), tie & (msg == 1))


def _relabel_index(order, n):
    N = 1 << n
    return np.array([sum(((j >> int(order[s])) & 1) << s for s in range(n)) for j in range(N)])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_permuted_graph_equals_relabelled_input(orc, seed):
    # BP on the graph with stage order sigma equals BP on the original graph
    # after relabelling rows by the bit permutation, bit for bit at every level
    rng = np.random.default_rng(seed)
    n, N = 7, 128
    code = orc.construct(N, 64, 2.0)
    sigma = rng.permutation(n).astype(np.int8)
    pi = _relabel_index(sigma, n)
    llr = rng.normal(0.8, 1.5, N).astype(np.float32)
    L1, R1 = orc.bp_run(llr, code.frozen, 6, order=sigma, alpha=0.9375)
    llr2 = np.zeros_like(llr)
    fr2 = np.zeros_like(code.frozen)
    llr2[pi] = llr
    fr2[pi] = code.frozen
    L2, R2 = orc.bp_run(llr2, fr2, 6, alpha=0.9375)
    np.testing.assert_array_equal(L1, L2[:, pi])
    np.testing.assert_array_equal(R1, R2[:, pi])


def test_fp32_tracks_fp64_early_iterations(orc):
    # per message |m32 - m64| <= 1e-5 max(|m64|, max|LLR|) over iterations 1..3:
    # a message is a signed sum of channel LLRs, so rounding error scales with
    # the frame's LLR magnitude even where the sum cancels to a small value
    code = orc.construct(1024, 512, 2.5)
    msg = synth.message_bits(4, 8, 512)
    _, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 2.5, 512, seed=4)
    for f in range(8):
        scale = float(np.abs(llr[f]).max())
        for it in (1, 2, 3):
            L32, R32 = orc.bp_run(llr[f], code.frozen, it, fp32=True)
            L64, R64 = orc.bp_run(llr[f], code.frozen, it, fp32=False)
            for A, B in ((L32, L64), (R32, R64)):
                fin = np.isfinite(B)
                assert np.array_equal(np.isfinite(A), fin)
                err = np.abs(A[fin] - B[fin]) / np.maximum(np.abs(B[fin]), scale)
                assert err.max() <= 1e-5


def test_decode_matches_bp_run_without_stop(orc):
    code = orc.construct(256, 144, 2.5, 16, 0x1021)
    msg = synth.message_bits(8, 6, code.K_msg)
    _, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 2.0, code.K_msg, seed=8)
    res = orc.decode(code, llr, orc.DecodeParams(max_iter=9, stop=orc.STOP_NONE), state=True)
    for f in range(6):
        L, R = orc.bp_run(llr[f], code.frozen, 9)
        np.testing.assert_array_equal(res.state[f, 0], L)
        np.testing.assert_array_equal(res.state[f, 1], R)


def test_crc_stop_semantics(orc):
    code = orc.construct(1024, 512, 2.5, 16, 0x1021)
    msg = synth.message_bits(11, 64, code.K_msg)
    u, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 2.75, code.K_msg, seed=11)
    p = orc.DecodeParams(max_iter=60, stop=orc.STOP_CRC, it_min=3)
    r = orc.decode(code, llr, p, threads=4)
    assert np.all(r.iters >= 3) and np.all(r.iters <= 60)
    stopped = r.iters < 60
    assert np.all(r.ok[stopped] == 1)
    # ok means the decided message satisfies its CRC
    for f in range(64):
        uh = r.msg_hat[f]
        full = orc.decode(code, llr[f:f + 1], orc.DecodeParams(max_iter=int(r.iters[f]),
                                                                stop=orc.STOP_NONE), soft=True)
        uh_all = (full.soft_u[0] < 0).astype(np.uint8)
        assert np.array_equal(uh_all[code.info_idx[:code.K_msg]], uh)
        c = orc.crc(uh, 16, 0x1021)
        tail = uh_all[code.info_idx[code.K_msg:]]
        assert (c == int("".join(map(str, tail)), 2)) == bool(r.ok[f])
    # the decoder should get most frames right at 2.75 dB
    assert (r.msg_hat != msg).any(1).mean() < 0.1


def test_g_stop_semantics(orc):
    code = orc.construct(64, 32, 2.0)
    msg = synth.message_bits(12, 200, 32)
    u, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 2.0, 32, seed=12)
    r = orc.decode(code, llr, orc.DecodeParams(max_iter=40, alpha=0.9375, stop=orc.STOP_G),
                   state=True)
    for f in range(200):
        L, R = r.state[f]
        uh = ((L[6] + R[6]) < 0).astype(np.uint8)
        xh = ((L[0] + R[0]) < 0).astype(np.uint8)
        assert bool(r.ok[f]) == np.array_equal(orc.polar_transform(uh), xh)
        if r.iters[f] < 40:
            assert r.ok[f] == 1


def _boxplus_decimal(x, y):
    """2 atanh(tanh(x/2) tanh(y/2)) in 150-digit decimal arithmetic."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 150
        def th(v):  # tanh(v/2) = (e^v - 1) / (e^v + 1)
            e = Decimal(v).exp()
            return (e - 1) / (e + 1)
        t = th(x) * th(y)
        if t == 0:
            return 0.0
        return float(((1 + t) / (1 - t)).ln())


_BOX_VALUES = [0.01, 0.5, 1.3, 7.0, 25.0, 40.0, 90.0]


@pytest.mark.parametrize("x", _BOX_VALUES + [-v for v in _BOX_VALUES])
@pytest.mark.parametrize("y", [0.25, 2.0, 7.0, 39.0, 40.0, -3.5, -88.0])
def test_exact_boxplus_against_high_precision(orc, x, y):
    # L(u0) of the N = 2 graph with both bits information is l0 boxplus l1;
    # both tanh factors round to 1 in FP64 beyond |v| of about 38, where the
    # function is still finite (40 boxplus 40 = 40 - ln 2 + ln(1 + e^-80))
    x32, y32 = float(np.float32(x)), float(np.float32(y))
    L, _ = orc.bp_run(np.array([x32, y32], np.float32), np.zeros(2, np.uint8), 1, fp32=False,
                      exact=True)
    want = _boxplus_decimal(x32, y32)
    assert math.isfinite(L[1, 0])
    assert L[1, 0] == pytest.approx(want, rel=1e-13, abs=1e-15)


def test_exact_boxplus_commutes_and_is_bounded(orc):
    # |x boxplus y| <= min(|x|, |y|), sign = product of the signs, symmetric
    rng = np.random.default_rng(4)
    for _ in range(50):
        v = rng.normal(0, 6, 2).astype(np.float32)
        L, _ = orc.bp_run(v, np.zeros(2, np.uint8), 1, fp32=False, exact=True)
        f = L[1, 0]
        assert abs(f) <= min(abs(float(v[0])), abs(float(v[1]))) + 1e-15
        assert np.sign(f) == np.sign(v[0]) * np.sign(v[1]) or f == 0
        L2, _ = orc.bp_run(np.array([v[1], v[0]], np.float32), np.zeros(2, np.uint8), 1,
                           fp32=False, exact=True)
        assert L2[1, 0] == f                      # commutative
