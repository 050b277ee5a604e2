"""Pins the oracle's cluster table (representative and intensity)."""
import math

import numpy as np
from scipy import stats as sps

from oracle.cluster import cluster_table, quantized_weights
from oracle.philox import TAG_REP, mulhi64, philox4x64


def vpls_from(rgb, pos=None):
    rgb = np.asarray(rgb, np.float32)
    n = rgb.shape[0]
    pos = np.zeros((n, 3), np.float32) if pos is None else np.asarray(pos, np.float32)
    return dict(x=pos[:, 0], y=pos[:, 1], z=pos[:, 2], nx=np.zeros(n, np.float32),
                ny=np.zeros(n, np.float32), nz=-np.ones(n, np.float32),
                ir=rgb[:, 0], ig=rgb[:, 1], ib=rgb[:, 2])


def test_singletons():
    rgb = np.random.default_rng(0).uniform(0, 1, (10, 3))
    v = vpls_from(rgb)
    rep, inten, lo, hi = cluster_table(v, np.arange(11, dtype=np.int32), np.arange(10, dtype=np.int32), 3)
    assert np.array_equal(rep, np.arange(10))
    assert np.array_equal(inten, rgb.astype(np.float32))


def test_two_member_cluster_by_hand():
    # member sums s = 0.75 and 0.25 -> weights 2^24 and floor(2^24 / 3) = 5592405
    v = vpls_from([[0.25, 0.25, 0.25], [0.125, 0.0625, 0.0625]], pos=[[0, 0, 1], [1, 2, 3]])
    off = np.array([0, 2], np.int32)
    mem = np.array([0, 1], np.int32)
    w = quantized_weights(np.array([0.75, 0.25]))
    assert list(w) == [1 << 24, 5592405]
    for seed in range(20):
        rep, inten, lo, hi = cluster_table(v, off, mem, seed)
        r0 = philox4x64((seed, 0), (0, 0, TAG_REP, 0))[0]
        u = mulhi64(r0, (1 << 24) + 5592405)
        assert rep[0] == (0 if u < (1 << 24) else 1)
        np.testing.assert_array_equal(inten[0], np.array([0.375, 0.3125, 0.3125], np.float32))
        np.testing.assert_array_equal(lo[0], [0, 0, 1])
        np.testing.assert_array_equal(hi[0], [1, 2, 3])


def test_intensity_is_exact_member_sum():
    rng = np.random.default_rng(4)
    rgb = rng.uniform(0, 1, (1000, 3)).astype(np.float32)
    v = vpls_from(rgb)
    perm = rng.permutation(1000).astype(np.int32)
    off = np.array([0, 300, 1000], np.int32)
    _, inten, _, _ = cluster_table(v, off, perm, 1)
    for c in range(2):
        mem = perm[off[c]:off[c + 1]]
        for ch in range(3):
            exact = math.fsum(float(x) for x in rgb[mem, ch])
            assert abs(float(inten[c, ch]) - exact) <= 0.5 * np.spacing(np.float32(exact)) * 1.0001


def test_representative_frequencies_follow_intensity():
    rgb = np.array([[0.1, 0.1, 0.1], [0.2, 0.2, 0.2], [0.4, 0.4, 0.4], [0.0, 0.0, 0.0]])
    v = vpls_from(rgb)
    off = np.array([0, 4], np.int32)
    mem = np.arange(4, dtype=np.int32)
    cnt = np.zeros(4)
    for seed in range(4000):
        rep, _, _, _ = cluster_table(v, off, mem, seed)
        cnt[rep[0]] += 1
    w = quantized_weights((rgb[:, 0].astype(np.float32).astype(np.float64) * 3))
    assert w[3] == 1                     # zero intensity still representable, weight 1
    res = sps.chisquare(cnt[:3], cnt[:3].sum() * w[:3] / w[:3].sum())
    assert res.pvalue > 1e-3
