"""Pins for the oracle's multi-trellis control (Sec. II-D, Sec. III, Eq. 2,
Algorithm 1, Table I)."""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "published_constants.json")))


def _frames(orc, N, K, c, poly, F, snr, seed):
    code = orc.construct(N, K, 2.5, c, poly)
    msg = synth.message_bits(seed, F, code.K_msg)
    _, x = orc.encode(code, msg)
    return code, msg, synth.awgn_llr(x, snr, code.K_msg, seed=seed)


def test_identity_pool_is_plain_bp(orc):
    code, msg, llr = _frames(orc, 1024, 512, 16, 0x1021, 24, 2.0, 1)
    base = orc.decode(code, llr, orc.DecodeParams(max_iter=80, stop=orc.STOP_CRC, it_min=3),
                      soft=True, threads=4)
    for mode, k in ((orc.PP_LASTK, 4), (orc.PP_FULL, 10)):
        r = orc.decode(code, llr, orc.DecodeParams(max_iter=80, stop=orc.STOP_CRC, it_min=3,
                                                   pp_mode=mode, k=k, T=5, Q=1, seed=7),
                       soft=True, threads=4)
        assert np.array_equal(r.iters, base.iters)
        assert np.array_equal(r.msg_hat, base.msg_hat)
        np.testing.assert_array_equal(r.soft_u, base.soft_u)


def test_no_event_before_T(orc):
    code, msg, llr = _frames(orc, 256, 144, 16, 0x1021, 8, 2.0, 2)
    p0 = orc.DecodeParams(max_iter=10, stop=orc.STOP_NONE)
    p1 = orc.DecodeParams(max_iter=10, stop=orc.STOP_NONE, pp_mode=orc.PP_LASTK, k=3, T=10, Q=8)
    a = orc.decode(code, llr, p0, state=True)
    b = orc.decode(code, llr, p1, state=True)
    np.testing.assert_array_equal(a.state, b.state)


@pytest.mark.parametrize("k,T", [(3, 5), (4, 10), (5, 5), (2, 3)])
def test_lastk_event_step(orc, k, T):
    # decode(T+2) = T plain iterations, reset of the inner levels of the permuted
    # range (paper levels n-k+2..n), one iteration on pool entry 1, ...
    code, msg, llr = _frames(orc, 1024, 512, 16, 0x1021, 3, 1.75, 3 + k)
    n = 10
    pool = orc.trellis_pool(n, k, 8, seed=21)
    p = orc.DecodeParams(max_iter=T + 1, stop=orc.STOP_NONE, pp_mode=orc.PP_LASTK, k=k, T=T,
                         Q=8, seed=21)
    r = orc.decode(code, llr, p, state=True)
    for f in range(3):
        L, R = orc.bp_run(llr[f], code.frozen, T)
        L[n - k + 1:n] = 0.0
        R[n - k + 1:n] = 0.0
        L, R = orc.bp_continue(L, R, 1, order=pool[1])
        np.testing.assert_array_equal(r.state[f, 0], L)
        np.testing.assert_array_equal(r.state[f, 1], R)


def test_pool_cycles_with_period_T(orc):
    # at iteration q*T the graph switches to pool entry q mod Q
    code, msg, llr = _frames(orc, 256, 144, 16, 0x1021, 2, 1.5, 9)
    n, k, T, Q = 8, 3, 2, 3
    pool = orc.trellis_pool(n, k, Q, seed=5)
    p = orc.DecodeParams(max_iter=7, stop=orc.STOP_NONE, pp_mode=orc.PP_LASTK, k=k, T=T, Q=Q,
                         seed=5)
    r = orc.decode(code, llr, p, state=True)
    for f in range(2):
        L, R = orc.bp_run(llr[f], code.frozen, 2)
        for q in (1, 2, 0):
            L[n - k + 1:n] = 0.0
            R[n - k + 1:n] = 0.0
            L, R = orc.bp_continue(L, R, 2 if q != 0 else 1, order=pool[q])
        np.testing.assert_array_equal(r.state[f, 0], L)
        np.testing.assert_array_equal(r.state[f, 1], R)


def test_full_permutation_keeps_only_channel_and_prior(orc):
    # Sec. II-D: after a full permutation only L_1 and R_{n+1} survive, so the
    # next iteration equals a fresh first iteration on the new graph
    code, msg, llr = _frames(orc, 512, 256, 16, 0x1021, 4, 1.5, 5)
    n, T = 9, 4
    pool = orc.trellis_pool(n, n, 8, seed=3)
    r = orc.decode(code, llr, orc.DecodeParams(max_iter=T + 1, stop=orc.STOP_NONE,
                                               pp_mode=orc.PP_FULL, T=T, Q=8, seed=3),
                   state=True)
    for f in range(4):
        L, R = orc.bp_run(llr[f], code.frozen, 1, order=pool[1])
        np.testing.assert_array_equal(r.state[f, 0], L)
        np.testing.assert_array_equal(r.state[f, 1, 1:], R[1:])


def test_fixed_pool_graphs_are_valid(orc):
    rng = np.random.default_rng(0)
    for n, k in ((10, 5), (8, 8), (6, 3)):
        N = 1 << n
        for order in orc.trellis_pool(n, k, 8, seed=1):
            u = rng.integers(0, 2, N).astype(np.uint8)
            assert np.array_equal(orc.graph_encode(np.tile(order, (N, 1)), u),
                                  orc.polar_transform(u))


@pytest.mark.parametrize("N,pr,pl,D,nmin", [(64, 6, 5, 4, 2), (256, 8, 7, 20, 3),
                                            (1024, 10, 9, 100, 15), (1024, 2, 6, 8, 4)])
def test_alg1_events_keep_graph_valid(orc, N, pr, pl, D, nmin):
    n = N.bit_length() - 1
    ords, nz, add, zeroed = orc.alg1_trace(N, pr, pl, D, nmin, seed=N + pr, n_events=25)
    rng = np.random.default_rng(1)
    for e in range(25):
        u = rng.integers(0, 2, N).astype(np.uint8)
        assert np.array_equal(orc.graph_encode(ords[e], u), orc.polar_transform(u))
        # N_zero = 2^m (rho_range - 1) nodes (per message type) are reset
        assert zeroed[e] == nz[e]
        if nz[e]:
            m_plus = [(2 ** m) * (r - 1) for r in range(2, pr + 1) for m in range(r, n + 1)]
            assert nz[e] in m_plus
        # Eq. 2
        assert add[e] == max(nmin, nz[e] // D)


def test_alg1_table1_short_budget_resets(orc):
    # Table I, N_it,max = 200: P_range = 2, P_level = 6, D = 8, N_min = 4 -> every
    # reset interval is one of {4, 8, 16}
    t = GOLD["table1_pp_bp_parameters"]["N1024_Nitmax200"]
    ords, nz, add, _ = orc.alg1_trace(1024, t["P_range"], t["P_level"], t["D"], t["N_min"],
                                      seed=4, n_events=200)
    assert set(add.tolist()) <= {4, 8, 16}
    assert set(nz.tolist()) <= {4, 8, 16, 32, 64, 128}
    assert len(set(add.tolist())) == 3


def test_alg1_full_range_reaches_full_permutation(orc):
    # Sec. IV: permuting the entire graph resets N (n-1) nodes
    # (first events of fresh decoders, while the graph is still the original)
    t = GOLD["table1_pp_bp_parameters"]["N1024_Nitmax20000"]
    full = GOLD["full_permutation_nzero"]["N1024"]
    firsts, adds = [], []
    for seed in range(60):
        _, nz, add, _ = orc.alg1_trace(1024, t["P_range"], t["P_level"], t["D"], t["N_min"],
                                       seed=seed, n_events=1)
        firsts.append(int(nz[0]))
        adds.append(int(add[0]))
    assert max(firsts) == full
    assert max(adds) == full // t["D"]


def test_alg1_subgraph_count(orc):
    # with rho_range = 2, rho_level = 1 (the N = 8 example of Fig. 3) there are
    # N / 2^2 = 2 subgraphs of 4 rows; the reset count is 4
    ords, nz, add, _ = orc.alg1_trace(8, 2, 1, 1, 1, seed=1, n_events=6)
    assert set(nz.tolist()) == {4}
    prev = np.tile(np.arange(3, dtype=np.int8), (8, 1))
    blocks = set()
    for o in ords:
        changed = np.nonzero((o != prev).any(1))[0]
        assert set(changed.tolist()) in ({0, 1, 2, 3}, {4, 5, 6, 7})
        blocks.add(int(changed[0]) // 4)
        # only stages 1..2 of the block change
        assert np.array_equal(o[:, 2], prev[:, 2])
        prev = o
    assert blocks == {0, 1}


def test_alg1_decode_runs(orc):
    code, msg, llr = _frames(orc, 256, 144, 16, 0x1021, 16, 2.5, 6)
    p = orc.DecodeParams(max_iter=200, stop=orc.STOP_CRC, it_min=3, pp_mode=orc.PP_ALG1,
                         P_range=8, P_level=7, D=20, N_min=5, seed=2)
    r = orc.decode(code, llr, p)
    assert np.all((r.iters >= 3) & (r.iters <= 200))
    assert (r.msg_hat != msg).any(1).mean() < 0.5


def test_fp32_fp64_fer_agree(orc):
    # frame error rates of the two precisions agree within a 95% Clopper-Pearson
    # interval (the decoders differ only through rounding)
    from scipy.stats import beta
    code, msg, llr = _frames(orc, 1024, 512, 16, 0x1021, 400, 2.25, 12)
    errs = {}
    for fp32 in (True, False):
        r = orc.decode(code, llr, orc.DecodeParams(max_iter=200, stop=orc.STOP_CRC, it_min=3,
                                                   pp_mode=orc.PP_LASTK, k=4, T=10, Q=8,
                                                   seed=1, fp32=fp32), threads=8)
        errs[fp32] = int((r.msg_hat != msg).any(1).sum())
    F = 400
    e = errs[False]
    lo = beta.ppf(0.025, e, F - e + 1) if e else 0.0
    hi = beta.ppf(0.975, e + 1, F - e)
    assert lo <= errs[True] / F <= hi


def _changed_rows(o, n):
    ident = np.arange(n, dtype=np.int8)
    return np.nonzero((o != ident).any(1))[0]


@pytest.mark.parametrize("N,pr,pl", [(64, 6, 5), (256, 8, 7), (1024, 10, 9), (1024, 2, 6)])
def test_alg1_r2_events_keep_graph_valid(orc, N, pr, pl):
    # reading R2 of Algorithm 1: each event restores the previous block and
    # permutes one aligned block of the ORIGINAL graph, so after every event the
    # schedule is the identity outside one block of 2^m rows
    n = N.bit_length() - 1
    ords, nz = orc.alg1_trace_r2(N, pr, pl, seed=N + pr, n_events=30)
    rng = np.random.default_rng(2)
    prev_sz = 0
    for e in range(30):
        u = rng.integers(0, 2, N).astype(np.uint8)
        assert np.array_equal(orc.graph_encode(ords[e], u), orc.polar_transform(u))
        rows = _changed_rows(ords[e], n)
        size = len(rows)
        m = size.bit_length() - 1
        assert size == 1 << m and m >= 2
        assert rows[0] % size == 0 and np.array_equal(rows, rows[0] + np.arange(size))
        # every row of the block carries the same stage order
        assert (ords[e][rows] == ords[e][rows[0]]).all()
        # nodes of levels rl..m-1 of the block: 2^m (rho_range - 1) of them,
        # plus those of the previous block that are not in this one
        assert nz[e] >= size
        if e == 0:
            assert nz[e] % size == 0 and 1 <= nz[e] // size <= pr - 1
        else:
            assert nz[e] <= prev_sz * (pr - 1) + size * (pr - 1)
        prev_sz = size


def test_alg1_r2_decode_runs_and_matches_plain_bp_before_first_event(orc):
    code, msg, llr = _frames(orc, 256, 144, 16, 0x1021, 16, 2.5, 6)
    base = dict(max_iter=200, stop=orc.STOP_CRC, it_min=3, P_range=8, P_level=7, D=20, N_min=5,
                seed=2)
    r2 = orc.decode(code, llr, orc.DecodeParams(pp_mode=orc.PP_ALG1_R2, **base))
    assert np.all((r2.iters >= 3) & (r2.iters <= 200))
    assert (r2.msg_hat != msg).any(1).mean() < 0.5
    # the first event comes after alg1_first_reset iterations: frames that stop
    # earlier are decoded exactly as plain BP decodes them
    plain = orc.decode(code, llr, orc.DecodeParams(pp_mode=orc.PP_NONE, max_iter=200,
                                                   stop=orc.STOP_CRC, it_min=3))
    first = min(max(256 * 7 // 20, 5), 100)
    early = plain.iters < first
    assert early.any()
    assert np.array_equal(r2.iters[early], plain.iters[early])
    assert np.array_equal(r2.msg_hat[early], plain.msg_hat[early])
