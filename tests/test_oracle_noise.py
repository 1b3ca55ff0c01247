"""Pins for the oracle's noise injection at the trellis events (the
future-work combination of Sec. V with the noise-aided BP of Table I): the
Gaussian draw against SplitMix64's published outputs and the Irwin-Hall
moments, the event step of the fixed schedules rebuilt from plain BP
iterations, the noisy channel level and the permuted graph, and Algorithm
1's channel level after a known number of events."""
import json
import os

import numpy as np
import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "published_constants.json")))


def _ih12(outputs):
    """Irwin-Hall sum of the twelve 16-bit fields of three 64-bit words."""
    s = sum((o >> (16 * k)) & 0xFFFF for o in outputs for k in range(4))
    return (s + 6) / 65536.0 - 6.0


def test_first_draw_is_built_from_published_splitmix_outputs(orc):
    # frame 0, event 0, row 0 with seed 0 starts the generator at state 0
    outs = [int(v, 16) for v in GOLD["splitmix64_seed0"]["outputs"]]
    assert orc.noise_gauss(0, 0, 0, 0) == _ih12(outs)


def test_draws_are_exact_and_have_irwin_hall_moments(orc):
    g = np.array([orc.noise_gauss(7, f, e, j) for f in range(4) for e in range(1, 6)
                  for j in range(0, 5000, 1)], np.float64)
    assert np.all(np.abs(g) < 6.0)
    assert np.all(g * 65536.0 == np.round(g * 65536.0))         # multiples of 2^-16
    n = g.size
    assert abs(g.mean()) < 5.0 / np.sqrt(n)
    assert abs(g.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    kurt = ((g - g.mean()) ** 4).mean() / g.var() ** 2          # Irwin-Hall(12): 3 - 1/10
    assert abs(kurt - 2.9) < 0.05
    # distinct (frame, event, row) give independent-looking draws
    assert len({orc.noise_gauss(1, 0, 1, j) for j in range(256)}) > 200


def _frames(orc, N, K, cw, poly, F, snr, seed):
    code = orc.construct(N, K, 2.5, cw, poly)
    msg = synth.message_bits(seed, F, code.K_msg)
    _, x = orc.encode(code, msg)
    return code, msg, synth.awgn_llr(x, snr, code.K_msg, seed=seed)


@pytest.mark.parametrize("Q,k", [(1, 0), (8, 4)])
def test_event_step_with_noise(orc, Q, k):
    # decode(T+1) = T plain iterations; at the event the channel level becomes
    # y + sigma g(frame, 1, j) in single precision (and with Q > 1 the inner
    # levels of the permuted range reset); one iteration on the event's graph
    code, msg, llr = _frames(orc, 256, 144, 16, 0x1021, 3, 2.0, 11)
    n, T, seed, sigma = 8, 4, 99, np.float32(0.6)
    p = orc.DecodeParams(max_iter=T + 1, stop=orc.STOP_NONE, pp_mode=orc.PP_LASTK, k=max(k, 2),
                         T=T, Q=Q, seed=seed, noise_sigma=float(sigma))
    r = orc.decode(code, llr, p, state=True)
    pool = orc.trellis_pool(n, max(k, 2), Q, seed=seed)
    for f in range(3):
        L, R = orc.bp_run(llr[f], code.frozen, T)
        g = np.array([orc.noise_gauss(seed, f, 1, j) for j in range(256)], np.float32)
        L[0] = (llr[f] + (sigma * g).astype(np.float32)).astype(np.float32)
        order = pool[1 % len(pool)]
        if len(pool) > 1:
            L[n - k + 1:n] = 0.0
            R[n - k + 1:n] = 0.0
        L, R = orc.bp_continue(L, R, 1, order=order)
        np.testing.assert_array_equal(r.state[f, 0], L)
        np.testing.assert_array_equal(r.state[f, 1], R)


def test_zero_sigma_is_the_plain_schedule(orc):
    code, msg, llr = _frames(orc, 128, 64, 8, 0x07, 20, 1.5, 3)
    kw = dict(max_iter=30, stop=orc.STOP_CRC, pp_mode=orc.PP_LASTK, k=3, T=5, Q=4, seed=2)
    a = orc.decode(code, llr, orc.DecodeParams(**kw), soft=True)
    b = orc.decode(code, llr, orc.DecodeParams(noise_sigma=0.0, **kw), soft=True)
    assert np.array_equal(a.msg_hat, b.msg_hat) and np.array_equal(a.iters, b.iters)
    c = orc.decode(code, llr, orc.DecodeParams(noise_sigma=0.6, **kw), soft=True)
    assert not np.array_equal(a.soft_u, c.soft_u)


@pytest.mark.parametrize("T0,d,E", [(3, 50, 1), (2, 4, 3)])
def test_algorithm1_channel_level_after_events(orc, T0, d, E):
    # Algorithm 1 with events after iterations T0, T0 + d, ... (D = 0 spaces
    # them by N_min = d): the channel level left at the end is y + sigma g of
    # the last event, e = E counting the frame's events, in single precision
    code, msg, llr = _frames(orc, 128, 80, 8, 0x07, 4, 1.5, 13)
    seed, sigma = 21, np.float32(0.6)
    max_iter = T0 + (E - 1) * d + 1
    p = orc.DecodeParams(max_iter=max_iter, stop=orc.STOP_NONE, pp_mode=orc.PP_ALG1, P_range=4,
                         P_level=3, D=0, N_min=d, first_reset=T0, seed=seed, noise_sigma=float(sigma))
    r = orc.decode(code, llr, p, state=True)
    for f in range(4):
        g = np.array([orc.noise_gauss(seed, f, E, j) for j in range(128)], np.float32)
        want = (llr[f] + (sigma * g).astype(np.float32)).astype(np.float32)
        np.testing.assert_array_equal(r.state[f, 0][0], want)


def test_algorithm1_noise_only_at_events(orc):
    # no event within the budget: the noise changes nothing; with events it does
    code, msg, llr = _frames(orc, 128, 80, 8, 0x07, 20, 1.5, 17)
    kw = dict(max_iter=30, stop=orc.STOP_CRC, pp_mode=orc.PP_ALG1, P_range=4, P_level=3, D=4, N_min=3,
              seed=5)
    a = orc.decode(code, llr, orc.DecodeParams(first_reset=40, **kw), soft=True)
    b = orc.decode(code, llr, orc.DecodeParams(first_reset=40, noise_sigma=0.6, **kw), soft=True)
    assert np.array_equal(a.soft_u, b.soft_u) and np.array_equal(a.iters, b.iters)
    c = orc.decode(code, llr, orc.DecodeParams(noise_sigma=0.6, **kw), soft=True)
    e = orc.decode(code, llr, orc.DecodeParams(**kw), soft=True)
    assert not np.array_equal(c.soft_u, e.soft_u)


def test_noise_is_rejected_without_events(orc):
    code, msg, llr = _frames(orc, 64, 40, 8, 0x07, 2, 2.0, 1)
    with pytest.raises(ValueError):
        orc.decode(code, llr, orc.DecodeParams(max_iter=5, noise_sigma=0.5))
