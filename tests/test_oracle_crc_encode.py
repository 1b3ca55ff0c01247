"""Pins for the oracle's CRC, polar transform, encoder and SplitMix64."""
import binascii
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "published_constants.json")))


def _bytes_to_bits(b: bytes):
    return np.array([(byte >> (7 - i)) & 1 for byte in b for i in range(8)], np.uint8)


def _poly_mod_crc(bits, width, poly):
    """Remainder of M(x) x^width modulo g(x) = x^width + poly, with Python ints."""
    g = (1 << width) | (poly & ((1 << width) - 1))
    m = 0
    for b in bits:
        m = (m << 1) | int(b)
    m <<= width
    deg = m.bit_length() - 1
    while deg >= width:
        m ^= g << (deg - width)
        deg = m.bit_length() - 1
    return m


def test_crc_check_values(orc):
    bits = _bytes_to_bits(b"123456789")
    assert orc.crc(bits, 16, 0x1021) == int(GOLD["crc_check_values"]["crc16_0x1021"], 16)
    assert orc.crc(bits, 24, 0x1864CFB) == int(GOLD["crc_check_values"]["crc24_0x864CFB"], 16)
    assert orc.crc(bits, 24, 0x864CFB) == int(GOLD["crc_check_values"]["crc24_0x864CFB"], 16)


def test_crc16_matches_binascii(orc):
    rng = np.random.default_rng(1)
    for L in [0, 1, 7, 62, 500]:
        b = rng.integers(0, 256, L, dtype=np.uint8).tobytes()
        assert orc.crc(_bytes_to_bits(b), 16, 0x1021) == binascii.crc_hqx(b, 0)


@pytest.mark.parametrize("width,poly", [(16, 0x1021), (24, 0x1864CFB), (8, 0x07), (3, 0x3)])
def test_crc_polynomial_division(orc, width, poly):
    rng = np.random.default_rng(width)
    for L in [1, 5, 33, 496, 2048]:
        bits = rng.integers(0, 2, L).astype(np.uint8)
        assert orc.crc(bits, width, poly) == _poly_mod_crc(bits, width, poly)


def test_crc_linear_and_zero(orc):
    rng = np.random.default_rng(5)
    a = rng.integers(0, 2, 496).astype(np.uint8)
    b = rng.integers(0, 2, 496).astype(np.uint8)
    assert orc.crc(np.zeros(496, np.uint8), 16, 0x1021) == 0
    assert orc.crc(a ^ b, 16, 0x1021) == orc.crc(a, 16, 0x1021) ^ orc.crc(b, 16, 0x1021)
    # message followed by its CRC leaves remainder zero
    c = orc.crc(a, 24, 0x1864CFB)
    tail = np.array([(c >> (23 - t)) & 1 for t in range(24)], np.uint8)
    assert orc.crc(np.concatenate([a, tail]), 24, 0x1864CFB) == 0


def _gn(n):
    F = np.array([[1, 0], [1, 1]], dtype=np.int64)
    g = np.array([[1]], dtype=np.int64)
    for _ in range(n):
        g = np.kron(g, F)
    return g % 2


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_polar_transform_bruteforce(orc, n):
    N = 1 << n
    g = _gn(n)
    rng = np.random.default_rng(n)
    us = (np.array([[(v >> i) & 1 for i in range(N)] for v in range(1 << N)], np.uint8)
          if N <= 8 else rng.integers(0, 2, (300, N)).astype(np.uint8))
    for u in us:
        assert np.array_equal(orc.polar_transform(u), (u.astype(np.int64) @ g % 2).astype(np.uint8))


def test_polar_transform_involution(orc):
    rng = np.random.default_rng(3)
    for N in [2, 64, 1024, 4096]:
        u = rng.integers(0, 2, N).astype(np.uint8)
        assert np.array_equal(orc.polar_transform(orc.polar_transform(u)), u)


def test_polar_transform_bit_permutation_invariance(orc):
    # relabelling rows by any bit permutation commutes with G_N
    rng = np.random.default_rng(4)
    n = 4
    N = 16
    for _ in range(20):
        tau = rng.permutation(n)
        perm = np.array([sum(((j >> b) & 1) << tau[b] for b in range(n)) for j in range(N)])
        u = rng.integers(0, 2, N).astype(np.uint8)
        v = np.zeros_like(u)
        v[perm] = u
        x = orc.polar_transform(u)
        y = np.zeros_like(x)
        y[perm] = x
        assert np.array_equal(orc.polar_transform(v), y)


def test_encode_places_message_and_crc(orc):
    code = orc.construct(1024, 512, 2.5, 16, 0x1021)
    rng = np.random.default_rng(6)
    msg = rng.integers(0, 2, (5, 496)).astype(np.uint8)
    u, x = orc.encode(code, msg)
    for f in range(5):
        assert np.all(u[f, code.frozen.astype(bool)] == 0)
        assert np.array_equal(u[f, code.info_idx[:496]], msg[f])
        c = orc.crc(msg[f], 16, 0x1021)
        assert np.array_equal(u[f, code.info_idx[496:]], [(c >> (15 - t)) & 1 for t in range(16)])
        assert np.array_equal(x[f], orc.polar_transform(u[f]))


def test_splitmix64_published(orc):
    want = [int(v, 16) for v in GOLD["splitmix64_seed0"]["outputs"]]
    assert orc.splitmix64_stream(0, 3) == want


@pytest.mark.parametrize("n,k,Q", [(10, 3, 8), (10, 4, 8), (10, 5, 8), (10, 10, 8), (6, 2, 8),
                                   (12, 5, 8), (3, 3, 6)])
def test_trellis_pool(orc, n, k, Q):
    pool = orc.trellis_pool(n, k, Q, seed=99)
    import math
    assert pool.shape == (min(Q, math.factorial(k)), n)
    assert list(pool[0]) == list(range(n))
    rows = {tuple(r) for r in pool}
    assert len(rows) == pool.shape[0]
    for r in pool[1:]:
        assert list(r[:n - k]) == list(range(n - k))
        assert sorted(r[n - k:]) == list(range(n - k, n))
        assert list(r) != list(range(n))
    # deterministic in the seed, different across seeds
    assert np.array_equal(pool, orc.trellis_pool(n, k, Q, seed=99))
