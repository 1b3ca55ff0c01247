"""Pins for the oracle's code construction (Sec. II-A): Bhattacharyya
recursion against brute-force successive-cancellation erasure probabilities on
the binary erasure channel, where the recursion is exact."""
import itertools
import math

import numpy as np
import pytest


def _gn(n):
    F = np.array([[1, 0], [1, 1]], dtype=np.int64)
    g = np.array([[1]], dtype=np.int64)
    for _ in range(n):
        g = np.kron(g, F)
    return g % 2


def _bitrev(i, n):
    return int(format(i, f"0{n}b")[::-1], 2) if n else 0


def _bec_sc_erasure(n, eps, order):
    """P(bit i ambiguous) for SC decoding of x = u G_N in the given order, by
    enumerating every erasure pattern and every completion of later bits."""
    N = 1 << n
    g = _gn(n)
    pos = {b: t for t, b in enumerate(order)}
    Z = np.zeros(N)
    for E in itertools.product([0, 1], repeat=N):
        pE = np.prod([eps if e else 1 - eps for e in E])
        seen = [k for k in range(N) if not E[k]]
        for i in range(N):
            later = [b for b in range(N) if pos[b] > pos[i]]
            amb = False
            for tail in itertools.product([0, 1], repeat=len(later)):
                v = np.zeros(N, np.int64)
                v[i] = 1
                v[later] = tail
                c = v @ g % 2
                if all(c[k] == 0 for k in seen):
                    amb = True
                    break
            if amb:
                Z[i] += pE
    return Z


@pytest.mark.parametrize("n,eps", [(1, 0.5), (2, 0.5), (2, 0.3), (3, 0.5), (3, 0.2)])
def test_bhattacharyya_equals_bec_sc_in_graph_order(orc, n, eps):
    # successive cancellation on the decoder's graph visits bits in bit-reversed order
    N = 1 << n
    order = [_bitrev(t, n) for t in range(N)]
    want = _bec_sc_erasure(n, eps, order)
    got = np.exp(orc.bhattacharyya(N, math.log(eps)))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def test_natural_order_differs(orc):
    # the natural SC order gives the mirrored vector; the oracle must not return it
    nat = _bec_sc_erasure(2, 0.5, [0, 1, 2, 3])
    np.testing.assert_allclose(nat, [0.9375, 0.5625, 0.4375, 0.0625])
    got = np.exp(orc.bhattacharyya(4, math.log(0.5)))
    np.testing.assert_allclose(got, [0.9375, 0.4375, 0.5625, 0.0625])


def test_bit_domination(orc):
    # if i's set bits are a subset of j's, channel j is at least as good
    N = 256
    lz = orc.bhattacharyya(N, -0.7)
    for i in range(N):
        for j in range(N):
            if i & j == i:
                assert lz[j] <= lz[i] + 1e-12


def test_construct_sets(orc):
    for N, K, snr in [(64, 32, 2.0), (1024, 512, 2.5), (256, 144, 2.5), (4096, 2072, 2.5)]:
        c = orc.construct(N, K, snr)
        assert c.info_idx.shape == (K,)
        assert np.all(np.diff(c.info_idx) > 0)
        assert c.frozen.sum() == N - K
        assert np.all(c.frozen[c.info_idx] == 0)
        lz = orc.construct_lnz(N, K, snr)
        # every information channel is at least as reliable as every frozen one
        assert lz[c.info_idx].max() <= lz[c.frozen.astype(bool)].min()
        # rate-1 position N-1 (all ones) is the best channel, 0 the worst
        assert (N - 1) in c.info_idx and 0 not in c.info_idx


def test_ties_go_to_larger_index(orc):
    # at z0 = 1 every channel has z = 1: the K largest indices are chosen
    c = orc.construct(32, 10, -math.inf)
    assert list(c.info_idx) == list(range(22, 32))


def test_recursion_single_step(orc):
    # N = 2: bit 0 degraded 2z - z^2, bit 1 upgraded z^2, for any z0
    for z in [0.9, 0.5, 1e-3]:
        got = np.exp(orc.bhattacharyya(2, math.log(z)))
        np.testing.assert_allclose(got, [2 * z - z * z, z * z], rtol=1e-12)
