"""Distribution pins of the oracle's random draws: the trellis pool's orders
(Sec. II-D, Sec. III: uniform over the non-identity orders of the permuted
stages) and Algorithm 1's rho_range, x, block and new order (Sec. III,
Algorithm 1: each drawn uniformly from its range).  Structure, range and
determinism pins elsewhere cannot see a biased shuffle (a Fisher-Yates draw
from [0, i) instead of [0, i] yields only cyclic orders, which still are
distinct non-identity orders); a chi-square test over many seeds does.  The
seeds are fixed, so each test is deterministic; the threshold p > 1e-4 leaves
a correct generator far from failing while any bias of a few percent per
class fails at these sample sizes."""
import itertools

import numpy as np
from scipy import stats

P_MIN = 1e-4


def _chi2_uniform(counts):
    counts = np.asarray(counts, np.float64)
    return stats.chisquare(counts).pvalue


def _perm_index(seq, base):
    """Index of the order `seq` of the values in `base` among all orders."""
    perms = list(itertools.permutations(sorted(base)))
    return perms.index(tuple(seq))


def test_pool_entry_uniform_over_nonidentity_orders(orc):
    n, k = 10, 4
    counts = np.zeros(24, np.int64)
    for seed in range(24 * 400):
        pool = orc.trellis_pool(n, k, 2, seed)
        counts[_perm_index(pool[1, n - k:].tolist(), range(n - k, n))] += 1
    ident = _perm_index(list(range(n - k, n)), range(n - k, n))
    assert counts[ident] == 0
    assert _chi2_uniform(np.delete(counts, ident)) > P_MIN


def test_pool_of_eight_covers_orders_uniformly(orc):
    # entries 1..7 of a pool of 8 (k = 4): each non-identity order appears
    # in a pool with probability 7/23, so pooled counts are uniform
    n, k = 12, 4
    counts = np.zeros(24, np.int64)
    for seed in range(3000):
        pool = orc.trellis_pool(n, k, 8, seed)
        assert len({tuple(r) for r in pool}) == 8
        for q in range(1, 8):
            counts[_perm_index(pool[q, n - k:].tolist(), range(n - k, n))] += 1
    ident = _perm_index(list(range(n - k, n)), range(n - k, n))
    assert counts[ident] == 0
    assert _chi2_uniform(np.delete(counts, ident)) > P_MIN


def test_pool_k3_second_entry_uniform(orc):
    n, k = 6, 3
    counts = np.zeros(6, np.int64)
    for seed in range(5 * 800):
        pool = orc.trellis_pool(n, k, 2, seed)
        counts[_perm_index(pool[1, n - k:].tolist(), range(n - k, n))] += 1
    assert counts[0] == 0          # identity is the first order in lexicographic order
    assert _chi2_uniform(counts[1:]) > P_MIN


def _first_draws(orc, N, P_range, P_level, n_seeds):
    out = []
    for seed in range(n_seeds):
        _, _, _, _, dr = orc.alg1_trace(N, P_range, P_level, 8, 4, seed + 1, 1, want_draws=True)
        out.append(dr[0])
    return np.array(out)


def test_alg1_draws_uniform_table1_long_set():
    import oracle as orc
    # the first event acts on the original graph, whose blocks all pass the
    # validity rule, so every draw there is accepted as drawn
    N, n, P_range, P_level = 1024, 10, 10, 9
    d = _first_draws(orc, N, P_range, P_level, 9000)
    rr, x, m, blk = d[:, 0], d[:, 1], d[:, 2], d[:, 3]
    assert rr.min() >= 2 and rr.max() <= P_range
    assert _chi2_uniform(np.bincount(rr, minlength=P_range + 1)[2:]) > P_MIN
    assert _chi2_uniform(np.bincount(x, minlength=P_level + 1)[1:]) > P_MIN
    rl = np.minimum(x, n - rr + 1)
    assert np.array_equal(m, rl + rr - 1)
    # the block, given m: 8 equiprobable bins over the N / 2^m blocks
    nb = N >> m
    sel = nb >= 8
    assert np.all(blk < nb) and np.all(blk >= 0)
    assert _chi2_uniform(np.bincount((blk[sel] * 8) // nb[sel], minlength=8)) > P_MIN
    # the new order, given rho_range = 3: uniform over the 5 non-identity orders
    counts = np.zeros(6, np.int64)
    for row, r, l in zip(d, rr, rl):
        if r == 3:
            counts[_perm_index(row[4:7].tolist(), range(l - 1, l + 2))] += 1
    assert counts[0] == 0
    assert _chi2_uniform(counts[1:]) > P_MIN


def test_alg1_draws_uniform_table1_200_set():
    import oracle as orc
    # P_range 2, P_level 6: rho_range is always 2 (a swap), x uniform on 1..6
    N, P_range, P_level = 1024, 2, 6
    d = _first_draws(orc, N, P_range, P_level, 6000)
    assert np.all(d[:, 0] == 2)
    assert _chi2_uniform(np.bincount(d[:, 1], minlength=7)[1:]) > P_MIN
    m, blk = d[:, 2], d[:, 3]
    assert np.array_equal(m, d[:, 1] + 1)
    nb = N >> m
    assert _chi2_uniform(np.bincount((blk * 8) // nb, minlength=8)) > P_MIN
    # the swapped pair is the two bits of stages x..x+1, in reversed order
    assert np.array_equal(d[:, 4], d[:, 1]) and np.array_equal(d[:, 5], d[:, 1] - 1)
