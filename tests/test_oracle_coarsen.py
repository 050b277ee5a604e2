"""Pins the oracle's per-slice light coarsening (Sec. 4): a hand-worked
four-leaf tree with closed-form entries, the merge order against a literal
scan of the available pairs and against the sorted-key prefix the GPU
computes, the error-bound mode against its definition, the pixel sets and
the node table."""
import dataclasses
import heapq
import math

import numpy as np
import pytest

from oracle import coarsen as C
from oracle import render as R
from oracle.philox import mulhi64, philox4x64


# ---------------------------------------------------------------- hand-worked tree
def _toy_scene():
    """Two Lambertian points (kd 0.5) facing up at (0,0,0) and (1,0,0); four
    VPLs facing down: L0 (0,0,1) I=1, L1 (0,0,2) I=2, L2 and L3 both at
    (1,0,1), I=1 and I=0.5; no occluders; tree ((L0, L1), (L2, L3))."""
    from scenegen import Scene, CONFIGS
    f = lambda *a: np.asarray(a, np.float32)
    pts = dict(px=f(0, 1), py=f(0, 0), pz=f(0, 0), nx=f(0, 0), ny=f(0, 0), nz=f(1, 1), kd_r=f(.5, .5),
               kd_g=f(.5, .5), kd_b=f(.5, .5), ks=f(0, 0), phong_e=f(1, 1), obj=np.zeros(2, np.int32))
    vpl = dict(x=f(0, 0, 1, 1), y=f(0, 0, 0, 0), z=f(1, 2, 1, 1), nx=f(0, 0, 0, 0), ny=f(0, 0, 0, 0),
               nz=f(-1, -1, -1, -1), ir=f(1, 2, 1, .5), ig=f(1, 2, 1, .5), ib=f(1, 2, 1, .5))
    sph = dict(cx=f(), cy=f(), cz=f(), r=f())
    i32 = lambda *a: np.asarray(a, np.int32)
    return Scene(cfg=CONFIGS["tiny"], seed=0, points=pts, vpls=vpl, spheres=sph, cut_offsets=i32(0, 1, 2, 3, 4),
                 cut_members=i32(0, 1, 2, 3), pt_offsets=i32(0, 2), pt_ids=i32(0, 1), cl_offsets=i32(0, 4),
                 cl_ids=i32(0, 1, 2, 3), rank=i32(1), tree_left=i32(0, 2, 4), tree_right=i32(1, 3, 5))


# unit-intensity Lambertian lighting S = kd / pi * cos_x cos_y / r^2 of the two
# points by the three distinct light positions, worked by hand
_S = {  # (point, light) -> S * pi / kd
    (0, 0): 1.0, (1, 0): 0.25,          # L0 at (0,0,1): r = 1 | r^2 = 2, cos = 1/sqrt2 each
    (0, 1): 0.25, (1, 1): 0.16,         # L1 at (0,0,2): r^2 = 4 | r^2 = 5, cos = 2/sqrt5 each
    (0, 2): 0.25, (1, 2): 1.0,          # L2, L3 at (1,0,1)
    (0, 3): 0.25, (1, 3): 1.0,
}


def _S_of(p, light):
    return 0.5 / math.pi * _S[(p, light)]


def test_hand_worked_four_leaf_tree():
    sc = _toy_scene()
    seed = 3
    tab = C.scene_table(sc, seed)
    # node table: I_f = I_a + I_b; the root holds all four lights
    np.testing.assert_array_equal(tab["intensity"][4], np.float32([3, 3, 3]))
    np.testing.assert_array_equal(tab["intensity"][5], np.float32([1.5, 1.5, 1.5]))
    np.testing.assert_array_equal(tab["intensity"][6], np.float32([4.5, 4.5, 4.5]))
    assert list(tab["height"][4:]) == [1, 1, 2] and list(tab["min_leaf"][4:]) == [0, 2, 0]
    for f in (4, 5, 6):
        assert tab["rep"][f] == tab["rep"][tab["kept"][f]]
        assert {tab["kept"][f], tab["dropped"][f]} == {tab["left"][f - 4], tab["right"][f - 4]}
    # eps(L_f) = max over both pixels of I_b |S(rep_b) - S(rep_a)| (one intensity per channel here)
    I = {x: float(tab["intensity"][x][0]) for x in range(7)}
    rep = {x: int(tab["rep"][x]) for x in range(7)}

    def eps(f):
        a, b = int(tab["kept"][f]), int(tab["dropped"][f])
        return max(I[b] * abs(_S_of(p, rep[b]) - _S_of(p, rep[a])) for p in (0, 1))

    p = R.Params(seed=seed)
    for n_max, merged_set in [(4, set()), (3, {5}), (2, {4, 5}), (1, {4, 5, 6})]:
        co = C.coarsen_slice(sc, tab, 0, seed, C.CoarsenParams(pixels=1 << 20), n_max, p)
        assert list(co["k"]) == [2, 2, 2, 2]                # every leaf sees both pixels
        assert set(co["merged"]) == merged_set, n_max
        assert co["n"] == n_max
        for f, e in co["eps"].items():
            assert abs(e - eps(f)) <= 1e-12, (f, e, eps(f))
        assert co["eps"][5] == 0.0                          # L2, L3 coincide: merging them is exact
        # the recursive cost: cost(f) = eps(f) + cost(dropped child); leaves cost 0
        if 6 in co["cost"]:
            d = int(tab["dropped"][6])
            assert abs(co["cost"][6] - (eps(6) + (eps(d) if d >= 4 else 0.0))) <= 1e-12
        # Omega1: both pixels of every column (each leaf saw both pixels)
        assert co["i1"].shape[0] == 2 * n_max
    # error-bound mode: only the exact merge is below 1e-9
    co = C.coarsen_slice(sc, tab, 0, seed, C.CoarsenParams(pixels=1 << 20, bound=1e-9), 4, p)
    assert co["merged"] == [5] and co["n"] == 3
    assert list(co["columns"]) == [0, 1, 5]


# ---------------------------------------------------------------- merge order on random trees
def _random_tree(rng, ng):
    """A random binary tree over ng leaves, split nodes numbered children first."""
    pool = list(range(ng))
    left, right = [], []
    nxt = ng
    while len(pool) > 1:
        a, b = rng.choice(len(pool), 2, replace=False)
        x, y = pool[a], pool[b]
        for i in sorted((a, b), reverse=True):
            pool.pop(i)
        left.append(x)
        right.append(y)
        pool.append(nxt)
        nxt += 1
    return np.array(left), np.array(right)


def _table(rng, ng):
    left, right = _random_tree(rng, ng)
    inten = rng.uniform(0.1, 1.0, (ng, 3)).astype(np.float32)
    z = np.zeros((ng, 3), np.float32)
    return C.node_table(np.arange(ng), inten, z, z, np.ones(ng, np.int64), left, right, int(rng.integers(1 << 30)))


def _literal_scan(tab, eps, n_max, bound, q):
    """Merge by scanning every available pair at every step (no heap)."""
    ng = tab["ng"]
    done = [x < ng for x in range(2 * ng - 1)]
    cost, eff = {}, {}
    merged = []
    count = ng
    while count > q:
        avail = []
        for k in range(ng - 1):
            f = ng + k
            if not done[f] and done[tab["left"][k]] and done[tab["right"][k]]:
                c = eps[f] + (cost[tab["dropped"][f]] if tab["dropped"][f] >= ng else 0.0)
                e = max([c] + [eff[ch] for ch in (tab["left"][k], tab["right"][k]) if ch >= ng])
                cost[f], eff[f] = c, e
                avail.append((e, int(tab["height"][f]), f))
        if not avail:
            break
        best = min(avail)
        if not (count > n_max or best[0] < bound):
            break
        merged.append(best[2])
        done[best[2]] = True
        count -= 1
    return merged


@pytest.mark.parametrize("seed", range(6))
def test_heap_order_matches_a_literal_scan(seed):
    rng = np.random.default_rng(seed)
    ng = int(rng.integers(5, 40))
    tab = _table(rng, ng)
    # eps with ties and zeros, as occluded or back-facing pairs give
    eps = {f: float(rng.choice([0.0, 0.5, 1.0, rng.uniform(0, 2)])) for f in range(ng, 2 * ng - 1)}
    for n_max in range(1, ng + 1):
        for bound, q in ((0.0, 1), (0.75, 1), (0.0, 3)):
            got, _, _ = C.greedy_merge(tab, lambda f: eps[f], n_max, bound, q)
            assert got == _literal_scan(tab, eps, n_max, bound, q), (n_max, bound, q)


@pytest.mark.parametrize("seed", range(6))
def test_merged_set_is_a_prefix_of_the_sorted_keys(seed):
    """The GPU's form: with every cost known, the merged nodes are the first L
    nodes in (eff, height, id) order, L = max(n_g - n_max, #{eff < bound})
    capped at n_g - q; every other node keeps both children."""
    rng = np.random.default_rng(100 + seed)
    ng = int(rng.integers(5, 60))
    tab = _table(rng, ng)
    eps = {f: float(rng.choice([0.0, 0.3, rng.uniform(0, 1)])) for f in range(ng, 2 * ng - 1)}
    cost, eff = {}, {}
    for f in range(ng, 2 * ng - 1):      # children first
        d = tab["dropped"][f]
        cost[f] = eps[f] + (cost[d] if d >= ng else 0.0)
        eff[f] = max([cost[f]] + [eff[c] for c in (tab["left"][f - ng], tab["right"][f - ng]) if c >= ng])
    keys = sorted((eff[f], int(tab["height"][f]), f) for f in range(ng, 2 * ng - 1))
    for n_max in (1, ng // 3 + 1, ng // 2 + 1, ng):
        for bound, q in ((0.0, 1), (0.31, 1), (0.0, 2)):
            L = min(ng - q, max(ng - n_max, sum(1 for k in keys if k[0] < bound)))
            got, _, _ = C.greedy_merge(tab, lambda f: eps[f], n_max, bound, q)
            assert sorted(got) == sorted(k[2] for k in keys[:max(0, L)]), (n_max, bound, q)


@pytest.mark.parametrize("seed", range(4))
def test_bound_mode_is_the_set_of_subtrees_below_the_bound(seed):
    """With no target count, a node is merged iff every merge in its subtree
    costs less than the bound (the order of merging does not matter)."""
    rng = np.random.default_rng(200 + seed)
    ng = int(rng.integers(5, 50))
    tab = _table(rng, ng)
    eps = {f: float(rng.uniform(0, 1)) for f in range(ng, 2 * ng - 1)}
    cost = {}
    for f in range(ng, 2 * ng - 1):
        d = tab["dropped"][f]
        cost[f] = eps[f] + (cost[d] if d >= ng else 0.0)
    below = C.leaf_sets(tab)
    for bound in (0.2, 0.6, 1.5):
        want = set()
        for f in range(ng, 2 * ng - 1):
            sub = [g for g in range(ng, 2 * ng - 1) if set(below[g]) <= set(below[f])]
            if all(cost[g] < bound for g in sub):
                want.add(f)
        got, _, _ = C.greedy_merge(tab, lambda f: eps[f], ng, bound, 1)
        assert set(got) == want, bound


# ---------------------------------------------------------------- pixel sets and node table
def test_pixel_set_counts_and_draws():
    rng = np.random.default_rng(7)
    inten = rng.uniform(0, 1, (50, 3)).astype(np.float32)
    K = 777
    k = C.leaf_quota(inten, K)
    t = C.total_intensity(inten)
    Q = np.maximum(1.0, np.floor(2.0 ** 24 * t / t.max()))
    np.testing.assert_array_equal(k, np.floor(K * Q / Q.sum()).astype(np.int64))
    assert k.sum() <= K
    for m in (1, 2, 3, 17, 64, 255, 300):
        for x in (0, 5):
            full = C.zeta_rows(9, 2, x, m, m)                 # the whole permutation
            assert sorted(full.tolist()) == list(range(m))
            assert np.array_equal(C.zeta_rows(9, 2, x, m, min(m, 7)), full[:min(m, 7)])
    a, b = C.zeta_rows(9, 2, 0, 200, 50), C.zeta_rows(9, 2, 1, 200, 50)
    assert not np.array_equal(a, b)                          # every leaf has its own permutation


def test_kept_child_draw_frequencies():
    """Over many split nodes with the same pair of intensities, the kept child
    is the left one with probability Q_l / (Q_l + Q_r)."""
    ng = 2
    inten = np.float32([[0.3, 0.3, 0.3], [0.1, 0.1, 0.1]])
    t = C.total_intensity(inten)
    ql, qr = C.quantize(t)
    hits = 0
    trials = 4000
    for f in range(trials):
        u = mulhi64(philox4x64((f, 0), (2, 0, C.TAG_TREE, 0))[0], ql + qr)
        tab = C.node_table(np.arange(ng), inten, np.zeros((2, 3), np.float32), np.zeros((2, 3), np.float32),
                           np.ones(2, np.int64), [0], [1], f)
        assert (tab["kept"][2] == 0) == (u < ql)
        hits += tab["kept"][2] == 0
    p = ql / (ql + qr)
    assert abs(hits / trials - p) < 4 * math.sqrt(p * (1 - p) / trials)


def test_no_merge_keeps_the_global_cut_and_its_draws():
    from scenegen import make_scene
    sc = make_scene("tiny", 2)
    tab = C.scene_table(sc, 2)
    p = R.Params(seed=2)
    co = C.coarsen_slice(sc, tab, 3, 2, C.CoarsenParams(pixels=2048), sc.n_clusters, p)
    assert co["merged"] == [] and co["n"] == sc.n_clusters
    assert list(co["columns"]) == list(range(sc.n_clusters))
    pairs = {(int(i), x) for x in range(sc.n_clusters) for i in co["zeta"][x]}
    assert pairs == set(zip(co["i1"].tolist(), co["j1"].tolist()))
    assert np.all(np.diff(co["i1"] * co["n"] + co["j1"]) > 0)      # row-major, each pair once
