"""Pins the oracle's sampling passes (first uniform pass, importance g(j),
second pass) against exhaustive enumeration, exact probabilities and
distribution tests."""
import itertools

import numpy as np
import pytest
from scipy import stats as sps

from oracle.philox import TAG_PASS2, mulhi64, philox4x64
from oracle.sampling import (column_stats, count_from_ppm, feistel, feistel_half_bits, importance,
                             pass1, pass2, weights_from_g)


def test_count_rounding_half_up():
    assert count_from_ppm(50000, 262144) == 13107          # 13107.2
    assert count_from_ppm(500000, 3) == 2                   # 1.5 -> 2
    assert count_from_ppm(250000, 2) == 1                   # 0.5 -> 1
    assert count_from_ppm(0, 10 ** 9) == 0
    assert count_from_ppm(10 ** 6, 12345) == 12345


@pytest.mark.parametrize("D", list(range(1, 300)) + [511, 512, 513, 1000, 2047, 2048, 2049, 4095, 4096])
def test_feistel_walk_is_a_bijection(D):
    h = feistel_half_bits(D)
    dom = 1 << (2 * h)
    assert dom >= D and dom < 4 * max(D, 4)
    x = np.arange(dom, dtype=np.uint64)
    y = feistel(x, 9, 3, h)
    assert np.array_equal(np.sort(y), x)                    # permutation of [0, 2^2h)
    i, j = pass1(9, 3, 1, D, 10 ** 6)                       # every entry: walk of 0..D-1
    e = i * D + j
    assert np.array_equal(np.sort(e), np.arange(D))


def test_pass1_count_distinct_in_range():
    m, n = 256, 1024
    i, j = pass1(1, 5, m, n, 50000)
    assert i.shape[0] == count_from_ppm(50000, m * n)
    e = i * n + j
    assert np.unique(e).shape[0] == e.shape[0]
    assert i.min() >= 0 and i.max() < m and j.min() >= 0 and j.max() < n


def test_pass1_marginals_uniform():
    m, n = 64, 96
    rows = np.zeros(m)
    cols = np.zeros(n)
    for s in range(40):
        i, j = pass1(7, s, m, n, 100000)
        rows += np.bincount(i, minlength=m)
        cols += np.bincount(j, minlength=n)
    assert sps.chisquare(rows).pvalue > 1e-3
    assert sps.chisquare(cols).pvalue > 1e-3


def test_pass1_depends_on_seed_and_slice():
    a = pass1(1, 0, 32, 32, 100000)[1]
    b = pass1(1, 1, 32, 32, 100000)[1]
    c = pass1(2, 0, 32, 32, 100000)[1]
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_column_stats_match_definitions():
    rng = np.random.default_rng(1)
    n = 7
    j = rng.integers(0, n - 1, 50)                          # last column never observed
    t = rng.uniform(0, 3, 50)
    cnt, mean, var, mn, mx = column_stats(j, t, n)
    for c in range(n):
        obs = t[j == c]
        assert cnt[c] == obs.shape[0]
        if obs.shape[0]:
            assert mn[c] == obs.min() and mx[c] == obs.max()
            np.testing.assert_allclose(mean[c], obs.mean(), rtol=1e-13)
            np.testing.assert_allclose(var[c], obs.var(), rtol=1e-9, atol=1e-14)
    g = importance(mn, mx, cnt)
    assert g[n - 1] == 0.0


def test_weights_hand_example():
    g = np.array([0.0, 1.0, 0.5, 1e-12, 0.25])
    w = weights_from_g(g)
    assert list(w) == [0, 1 << 24, 1 << 23, 1, 1 << 22]
    assert list(weights_from_g(np.zeros(4))) == [1, 1, 1, 1]


def test_mixed_weights_hand_example():
    """g(j) + mix mean g: with g = (0, 1, 2, 4) the paper's weights are
    2^20 (0, 4, 8, 16), their sum 28 2^20, and at mix = 1 the offset is
    c = floor(28 2^20 / 4) = 7 2^20; then w_j = floor(2^24 (q_j + c) / (2^24 + c))
    = floor(2^24 k_j / 23) with k = (7, 11, 15, 23)."""
    g = np.array([0.0, 1.0, 2.0, 4.0])
    w = weights_from_g(g, 1.0)
    assert list(w) == [117440512 // 23, 184549376 // 23, 251658240 // 23, 1 << 24]
    assert list(w) == [5106109, 8023885, 10941662, 16777216]
    # mix 0 is the paper's rule; +inf the uniform density
    assert np.array_equal(weights_from_g(g, 0.0), weights_from_g(g))
    assert list(weights_from_g(g, np.inf)) == [1, 1, 1, 1]
    # a small mix whose offset rounds to zero leaves the paper's weights
    assert np.array_equal(weights_from_g(g, 1e-9), weights_from_g(g))


def test_mixed_weights_properties():
    rng = np.random.default_rng(4)
    g = rng.exponential(1.0, 700) * (rng.uniform(0, 1, 700) < 0.7)
    q = weights_from_g(g).astype(np.float64)
    prev = None
    for mix in (0.1, 0.3, 1.0, 3.0, 100.0, 1e6):
        w = weights_from_g(g, mix).astype(np.float64)
        assert (w >= 1).all() and (w <= 2 ** 24).all()
        order = np.argsort(g, kind="stable")
        assert (np.diff(w[order]) >= 0).all()                 # monotone in g
        # the density is g + mix mean g (up to the integer rounding)
        p = w / w.sum()
        want = (q + mix * q.mean()) / (q + mix * q.mean()).sum()
        np.testing.assert_allclose(p, want, rtol=1e-5, atol=1e-9)
        spread = w.max() / w.min()
        if prev is not None:
            assert spread <= prev                              # flatter as mix grows
        prev = spread
    assert weights_from_g(g, 1e6).min() / weights_from_g(g, 1e6).max() > 0.999
    for bad in (-1.0, np.nan):
        with pytest.raises(ValueError):
            weights_from_g(g, bad)


def test_pass2_first_attempt_by_hand():
    # recompute attempt 0 by hand from the generator and compare
    m, n = 5, 4
    w = np.array([3, 0, 1, 4], dtype=np.uint64)
    taken = np.zeros(m * n, bool)
    i2, j2, short = pass2(77, 2, m, n, 0, 50000, w, taken)   # N2 = 1
    r0, r1, _, _ = philox4x64((77, 2), (0, 0, TAG_PASS2, 0))
    u = mulhi64(r0, 8)
    jj = 0 if u < 3 else (2 if u < 4 else 3)
    ii = mulhi64(r1, m)
    assert (i2[0], j2[0]) == (ii, jj) and not short


def test_pass2_exact_acceptance_probabilities():
    """2 x 3 slice, entry (0, 0) taken by the first pass, N2 = 1: the accepted
    entry has probability p(e) / (1 - p(0, 0)), p(i, j) = w_j / W / m."""
    m, n = 2, 3
    w = np.array([2, 1, 1], dtype=np.uint64)
    W = 4.0
    taken = np.zeros(m * n, bool)
    taken[0] = True
    p = np.array([[w[j] / W / m for j in range(n)] for i in range(m)]).ravel()
    expect = p.copy()
    expect[0] = 0.0
    expect /= expect.sum()
    trials = 20000
    freq = np.zeros(m * n)
    for seed in range(trials):
        i2, j2, _ = pass2(seed, 0, m, n, 1, 166667, w, taken)
        assert i2.shape[0] == 1
        freq[i2[0] * n + j2[0]] += 1
    assert freq[0] == 0
    res = sps.chisquare(freq[1:], expect[1:] * trials)
    assert res.pvalue > 1e-3


def test_pass2_column_frequency_follows_weights():
    m, n = 4096, 8                                        # collisions negligible
    w = np.array([1, 2, 3, 4, 0, 8, 16, 2], dtype=np.uint64)
    taken = np.zeros(m * n, bool)
    i2, j2, short = pass2(3, 1, m, n, 0, 30000, w, taken)
    assert not short
    cnt = np.bincount(j2, minlength=n)
    assert cnt[4] == 0
    nz = w > 0
    res = sps.chisquare(cnt[nz], cnt.sum() * w[nz] / w.sum())
    assert res.pvalue > 1e-3


def test_pass2_no_duplicates_and_disjoint_from_pass1():
    m, n = 32, 64
    i1, j1 = pass1(5, 0, m, n, 200000)
    taken = np.zeros(m * n, bool)
    taken[i1 * n + j1] = True
    w = np.arange(1, n + 1, dtype=np.uint64)
    i2, j2, short = pass2(5, 0, m, n, i1.shape[0], 300000, w, taken)
    e2 = i2 * n + j2
    assert not short
    assert np.unique(e2).shape[0] == e2.shape[0]
    assert not taken[e2].any()


def test_pass2_full_rate_takes_the_rest_row_major():
    m, n = 6, 5
    i1, j1 = pass1(1, 0, m, n, 300000)
    taken = np.zeros(m * n, bool)
    taken[i1 * n + j1] = True
    i2, j2, short = pass2(1, 0, m, n, i1.shape[0], 10 ** 6, np.ones(n, np.uint64), taken)
    e2 = i2 * n + j2
    assert np.array_equal(e2, np.nonzero(~taken)[0])
    assert np.array_equal(np.sort(np.concatenate([i1 * n + j1, e2])), np.arange(m * n))


def test_pass2_shortfall():
    # all weight on column 0 with only 3 rows, 5 entries requested
    m, n = 3, 10
    w = np.zeros(n, np.uint64)
    w[0] = 1
    taken = np.zeros(m * n, bool)
    i2, j2, short = pass2(1, 0, m, n, 0, 166667, w, taken)
    assert short and i2.shape[0] == 3 and set(j2) == {0}


def test_pass2_sequential_semantics_by_enumeration():
    """Simulate the sequential rule directly from the generator for a few
    attempts and compare every accepted entry and its order."""
    m, n = 3, 4
    w = np.array([1, 5, 0, 2], dtype=np.uint64)
    P = np.cumsum(w)
    taken = np.zeros(m * n, bool)
    taken[[1, 6]] = True
    got_i, got_j, _ = pass2(11, 4, m, n, 2, 400000, w, taken)   # N2 = round(0.4 * 12) = 5
    seen = set([1, 6])
    acc = []
    for t in itertools.count():
        r0, r1, _, _ = philox4x64((11, 4), (t, 0, TAG_PASS2, 0))
        j = int(np.searchsorted(P, mulhi64(r0, int(P[-1])), side="right"))
        i = mulhi64(r1, m)
        if i * n + j not in seen:
            seen.add(i * n + j)
            acc.append((i, j))
        if len(acc) == 5:
            break
    assert list(zip(got_i.tolist(), got_j.tolist())) == acc
