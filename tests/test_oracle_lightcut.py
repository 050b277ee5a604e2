"""Pins the oracle's global light cut (Sec. 3 step 1, Sec. 6): the error
bound's closed forms and its upper-bound property by brute force over a
node's VPLs, the estimate against the brute-force column sum, a hand-worked
four-VPL frame (both pairs' worst ratios and the cut for every eps and cap),
and the cut's structure on random scenes."""
import math

import numpy as np
import pytest

import scenegen
from oracle import lightcut as LC
from oracle import render as R
from oracle.shading import entries, point_arrays


def _scene(pts, vpls):
    i32 = lambda *a: np.asarray(a, np.int32)
    sph = {k: np.zeros(0, np.float32) for k in ("cx", "cy", "cz", "r")}
    return scenegen.Scene(cfg=scenegen.CONFIGS["tiny"], seed=0, points=pts, vpls=vpls, spheres=sph,
                          cut_offsets=i32(0), cut_members=i32(), pt_offsets=i32(0), pt_ids=i32(),
                          cl_offsets=i32(0), cl_ids=i32(), rank=i32())


def _points(p, n, kd, ks=None, pe=None):
    f32 = lambda a: np.asarray(a, np.float32)
    p, n, kd = np.asarray(p, float), np.asarray(n, float), np.asarray(kd, float)
    m = p.shape[0]
    return dict(px=f32(p[:, 0]), py=f32(p[:, 1]), pz=f32(p[:, 2]), nx=f32(n[:, 0]), ny=f32(n[:, 1]),
                nz=f32(n[:, 2]), kd_r=f32(kd[:, 0]), kd_g=f32(kd[:, 1]), kd_b=f32(kd[:, 2]),
                ks=f32(np.zeros(m) if ks is None else ks), phong_e=f32(np.ones(m) if pe is None else pe),
                obj=np.zeros(m, np.int32))


def _vpls(y, ny, I):
    f32 = lambda a: np.asarray(a, np.float32)
    y, ny, I = np.asarray(y, float), np.asarray(ny, float), np.asarray(I, float)
    return dict(x=f32(y[:, 0]), y=f32(y[:, 1]), z=f32(y[:, 2]), nx=f32(ny[:, 0]), ny=f32(ny[:, 1]),
                nz=f32(ny[:, 2]), ir=f32(I[:, 0]), ig=f32(I[:, 1]), ib=f32(I[:, 2]))


# ------------------------------------------------------------------ the bound
@pytest.mark.parametrize("d", [0.7, 0.03])
@pytest.mark.parametrize("phong", [False, True])
def test_bound_equals_the_entry_of_a_vpl_on_the_normal(d, phong):
    """A VPL on the pixel's normal facing it: every cosine is 1, the Phong
    lobe is at its peak (viewer on the normal), so bound = entry exactly,
    r_min clamp included (d = 0.03 < r_min)."""
    x = np.array([[0.3, 0.2, 0.1]])
    n = np.array([[0.0, 0.0, 1.0]])
    kd = np.array([[0.6, 0.4, 0.2]])
    ks, pe = (np.array([0.3]), np.array([40.0])) if phong else (np.zeros(1), np.ones(1))
    y = x + np.array([[0.0, 0.0, d]])
    I = np.array([[1.5, 2.0, 0.5]])
    b = LC.bound(x, n, kd, ks, pe, y, y, I, r_min=0.05)
    f = kd / math.pi + (ks * (pe + 2.0) / (2.0 * math.pi))[:, None]
    want = (f * I).sum() / max(d * d, 0.05 ** 2)
    assert b[0] == pytest.approx(want, rel=1e-13)


def test_bound_is_zero_below_the_horizon_and_positive_above():
    x = np.zeros((2, 3))
    n = np.array([[0.0, 0.0, 1.0]] * 2)
    kd = np.full((2, 3), 0.5)
    lo = np.array([[-1.0, -1.0, -2.0], [-1.0, -1.0, -2.0]])
    hi = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1e-3]])     # top face at the plane / just above it
    b = LC.bound(x, n, kd, np.zeros(2), np.ones(2), lo, hi, np.ones((2, 3)), r_min=0.05)
    assert b[0] == 0.0 and b[1] > 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bound_holds_for_every_node_by_brute_force(seed):
    """For random VPLs (any orientation), pixels (some Phong) and every node
    of the full light tree: the bound is at least the node's true
    unoccluded contribution (each VPL its own light) and at least its
    representative's."""
    rng = np.random.default_rng(seed)
    nv, m = 24, 16
    y = rng.uniform(-1, 1, (nv, 3))
    ny = rng.normal(size=(nv, 3))
    ny /= np.linalg.norm(ny, axis=1, keepdims=True)
    vp = _vpls(y, ny, rng.uniform(0, 1, (nv, 3)))
    p = rng.uniform(-1.5, 1.5, (m, 3))
    nn = rng.normal(size=(m, 3))
    nn /= np.linalg.norm(nn, axis=1, keepdims=True)
    pts = _points(p, nn, rng.uniform(0.1, 0.9, (m, 3)), ks=np.where(rng.uniform(size=m) < 0.5, 0.2, 0.0),
                  pe=rng.uniform(5, 60, m))
    perm, left, right = scenegen.full_light_tree(y)
    tab = LC.light_tree_table(vp, perm, left, right, seed)
    Y = np.stack([vp["x"], vp["y"], vp["z"]], 1).astype(np.float64)
    NY = np.stack([vp["nx"], vp["ny"], vp["nz"]], 1).astype(np.float64)
    IY = np.stack([vp["ir"], vp["ig"], vp["ib"]], 1).astype(np.float64)
    x, n, kd, ks, pe, wo = point_arrays(pts, np.arange(m))
    lo_leaf = np.arange(2 * nv - 1)
    for f in range(2 * nv - 1):
        members = perm[tab["min_leaf"][f]:tab["min_leaf"][f] + tab["members"][f]]
        lo = np.repeat(tab["lo"][f][None].astype(np.float64), m, 0)
        hi = np.repeat(tab["hi"][f][None].astype(np.float64), m, 0)
        I = np.repeat(tab["intensity"][f][None].astype(np.float64), m, 0)
        b = LC.bound(x, n, kd, ks, pe, lo, hi, I, r_min=0.05)
        true = np.zeros(m)
        for j in members:
            A, _, _ = entries(x, n, kd, ks, pe, wo, np.repeat(Y[j][None], m, 0), np.repeat(NY[j][None], m, 0),
                              np.repeat(IY[j][None], m, 0), None, r_min=0.05, with_visibility=False)
            true += A.sum(axis=1)
        rep = tab["rep"][f]
        A, _, _ = entries(x, n, kd, ks, pe, wo, np.repeat(Y[rep][None], m, 0), np.repeat(NY[rep][None], m, 0), I,
                          None, r_min=0.05, with_visibility=False)
        assert (b >= true * (1 - 1e-12)).all(), f
        assert (b >= A.sum(axis=1) * (1 - 1e-12)).all(), f
    del lo_leaf


def test_estimate_of_all_single_vpls_is_the_brute_force_sum():
    rng = np.random.default_rng(5)
    nv, m = 40, 12
    y = rng.uniform(-1, 1, (nv, 3)) + np.array([0, 0, 2.0])
    ny = np.tile([0.0, 0.0, -1.0], (nv, 1))
    vp = _vpls(y, ny, rng.uniform(0, 1, (nv, 3)))
    p = np.c_[rng.uniform(-1, 1, (m, 2)), np.zeros(m)]
    pts = _points(p, np.tile([0.0, 0.0, 1.0], (m, 1)), rng.uniform(0.1, 0.9, (m, 3)),
                  ks=np.full(m, 0.2), pe=np.full(m, 20.0))
    perm, left, right = scenegen.full_light_tree(y)
    tab = LC.light_tree_table(vp, perm, left, right, 0)
    est = LC.estimate(pts, np.arange(m), vp, tab, np.arange(nv), r_min=0.05)
    ref = R.brute_force(_scene(pts, vp), R.Params(), point_ids=np.arange(m)).sum(axis=1)
    np.testing.assert_allclose(est, ref, rtol=1e-12)


# ------------------------------------------------------- hand-worked frame
def _four_vpl_frame():
    """Pixels x1 = (0,0,0), x2 = (0,4,0) facing +z, Lambertian, kd 1.  VPLs
    facing -z with red intensity 1: A (-1,0,1), B (1,0,1) near x1, C (-0.5,4,1),
    D (0.5,4,1) near x2.  The tree splits the root along y into the pairs
    P1 = {A, B} (node 5) and P2 = {C, D} (node 4), each along x; root node 6."""
    pts = _points([[0, 0, 0], [0, 4, 0]], [[0, 0, 1]] * 2, [[1, 1, 1]] * 2)
    vp = _vpls([[-1, 0, 1], [1, 0, 1], [-0.5, 4, 1], [0.5, 4, 1]], [[0, 0, -1]] * 4, [[1, 0, 0]] * 4)
    return pts, vp


# By hand (unit red intensity, kd / pi = 1 / pi, G = cos_x cos_y / r^2 = h^2 / r^4 at height h = 1):
#   x1: G(A) = G(B) = 1/4 (r^2 = 2), G(C) = G(D) = 1/17.25^2 (r^2 = 0.25 + 16 + 1)
#   x2: G(A) = G(B) = 1/18^2, G(C) = G(D) = 1/1.25^2 = 0.64
# With the cut {P1, P2} (reps irrelevant by symmetry, I = 2 each):
#   est(x1) = (2/pi)(1/4 + 1/17.25^2), est(x2) = (2/pi)(0.64 + 1/18^2)
# Bounds (2/pi) G_ub: a pair's box straight above the pixel has d_min = 1,
# cosine bound 1 -> G_ub = 1; the other pair's box is at d_min^2 = 4^2 + 1 = 17
# with h = 1 -> cosine bound 1/sqrt(17), G_ub = 17^-1.5.
_EST1 = 0.25 + 1.0 / 17.25 ** 2
_EST2 = 0.64 + 1.0 / 18.0 ** 2
RHO_P1 = max(1.0 / _EST1, 17.0 ** -1.5 / _EST2)     # = 3.946943...
RHO_P2 = max(17.0 ** -1.5 / _EST1, 1.0 / _EST2)     # = 1.555001...


def test_hand_worked_frame_tree_layout():
    pts, vp = _four_vpl_frame()
    perm, left, right = scenegen.full_light_tree(np.stack([vp["x"], vp["y"], vp["z"]], 1))
    assert list(perm) == [0, 1, 2, 3]
    assert list(left) == [2, 0, 5] and list(right) == [3, 1, 4]


@pytest.mark.parametrize("eps,cap,cut,offsets,al,ar", [
    (400.0, 64, [6], [0, 4], [], []),
    (5.0, 64, [5, 4], [0, 2, 4], [0], [1]),
    (2.0, 64, [0, 1, 4], [0, 1, 2, 4], [0, 3], [1, 2]),
    (1.0, 64, [0, 1, 2, 3], [0, 1, 2, 3, 4], [2, 0, 5], [3, 1, 4]),
    (1.0, 3, [0, 1, 4], [0, 1, 2, 4], [0, 3], [1, 2]),     # room for one split: the larger rho (P1)
    (1.0, 2, [5, 4], [0, 2, 4], [0], [1]),
    (1.0, 1, [6], [0, 4], [], []),
])
def test_hand_worked_frame_cut(eps, cap, cut, offsets, al, ar):
    pts, vp = _four_vpl_frame()
    perm, left, right = scenegen.full_light_tree(np.stack([vp["x"], vp["y"], vp["z"]], 1))
    out = LC.lightcut(pts, vp, perm, left, right, [0, 1], eps, cap, r_min=0.05, seed=7)
    assert list(out["cut"]) == cut
    assert list(out["offsets"]) == offsets
    assert list(out["above_left"]) == al and list(out["above_right"]) == ar
    assert out["ambiguous"] == 0
    rep = out["table"]["rep"][6]
    # root: est = (4/pi) G(x, rep), bound = 4/pi at both pixels (its box is over both)
    assert out["rho"][6] == pytest.approx(324.0 if rep in (0, 1) else 17.25 ** 2, rel=1e-12)
    if 5 in out["rho"]:
        assert out["rho"][5] == pytest.approx(RHO_P1, rel=1e-12)
        assert out["rho"][4] == pytest.approx(RHO_P2, rel=1e-12)
    assert RHO_P1 == pytest.approx(3.9469430, rel=1e-7) and RHO_P2 == pytest.approx(1.5550010, rel=1e-7)


# ------------------------------------------------------------ structure
def _random_frame(seed, nv=200, m=64):
    rng = np.random.default_rng(seed)
    y = np.c_[rng.uniform(0, 2, nv), rng.uniform(0, 1, nv), rng.uniform(0.3, 1.0, nv)]
    d = rng.normal(size=(nv, 3))
    d[:, 2] = np.abs(d[:, 2])
    ny = -d / np.linalg.norm(d, axis=1, keepdims=True)
    vp = _vpls(y, ny, rng.uniform(0, 1, (nv, 3)))
    p = np.c_[rng.uniform(0, 2, m), rng.uniform(0, 1, m), np.zeros(m)]
    pts = _points(p, np.tile([0.0, 0.0, 1.0], (m, 1)), rng.uniform(0.2, 0.9, (m, 3)),
                  ks=np.where(rng.uniform(size=m) < 0.5, 0.2, 0.0), pe=rng.uniform(10, 100, m))
    perm, left, right = scenegen.full_light_tree(y)
    return pts, vp, perm, left, right


@pytest.mark.parametrize("eps,cap", [(0.02, 10_000), (0.1, 10_000), (0.02, 40), (0.5, 7)])
def test_cut_is_a_partition_within_the_cap_and_passes_its_tests(eps, cap):
    pts, vp, perm, left, right = _random_frame(11)
    out = LC.lightcut(pts, vp, perm, left, right, np.arange(64), eps, cap, seed=3)
    n = perm.shape[0]
    tab = out["table"]
    cut, off = out["cut"], out["offsets"]
    assert len(cut) <= cap and off[0] == 0 and off[-1] == n
    for k, f in enumerate(cut):      # contiguous, in order, covering every leaf once
        assert tab["min_leaf"][f] == off[k] and tab["members"][f] == off[k + 1] - off[k]
    capped = sum(lv["failing"] > lv["split"] for lv in out["levels"])
    for f in cut:
        if f >= n and f in out["rho"] and not capped:
            assert out["rho"][f] <= eps
    # the tree above the cut: valid coarsening layout over the cut's clusters
    ng = len(cut)
    al, ar = out["above_left"], out["above_right"]
    assert al.shape[0] == ng - 1
    parent = -np.ones(2 * ng - 1, int)
    for k in range(ng - 1):
        for c in (al[k], ar[k]):
            assert 0 <= c < ng + k and parent[c] < 0
            parent[c] = ng + k
    assert (parent[:-1] >= 0).all()


def test_eps_zero_splits_to_single_vpls_and_huge_eps_keeps_the_root():
    pts, vp, perm, left, right = _random_frame(4, nv=60, m=16)
    n = perm.shape[0]
    out = LC.lightcut(pts, vp, perm, left, right, np.arange(16), 0.0, 10 ** 6)
    assert list(out["cut"]) == list(range(n))
    out = LC.lightcut(pts, vp, perm, left, right, np.arange(16), np.inf, 10 ** 6)   # b / 0 = inf fails any finite eps
    assert list(out["cut"]) == [2 * n - 2]
    out = LC.lightcut(pts, vp, perm, left, right, np.zeros(0, np.int64), 0.0, 10 ** 6)
    assert list(out["cut"]) == [2 * n - 2]     # no pixel to bound: nothing fails


def test_single_vpl():
    pts, vp, perm, left, right = _random_frame(2, nv=1, m=4)
    out = LC.lightcut(pts, vp, perm, left, right, np.arange(4), 0.0, 5)
    assert list(out["cut"]) == [0] and list(out["offsets"]) == [0, 1] and out["above_left"].size == 0


@pytest.mark.parametrize("y", [[3.0, 0.0, 1.0], [-0.4, 0.9, 0.2], [0.01, 0.0, 0.02]])
def test_bound_equals_the_entry_of_a_lambertian_vpl_facing_the_pixel(y):
    """A single VPL (box = its point) whose normal points at the pixel: the
    light-side cosine is 1 and h / d_min is the pixel-side cosine itself,
    so for a Lambertian pixel bound = entry, at any angle above the horizon."""
    x = np.array([[0.0, 0.0, 0.0]])
    n = np.array([[0.0, 0.0, 1.0]])
    kd = np.array([[0.7, 0.5, 0.3]])
    Y = np.asarray([y], float)
    w = Y / np.linalg.norm(Y)
    I = np.array([[0.8, 1.1, 0.4]])
    b = LC.bound(x, n, kd, np.zeros(1), np.ones(1), Y, Y, I, r_min=0.05)
    A, _, _ = entries(x, n, kd, np.zeros(1), np.ones(1), np.array([[0.0, 0.0, 1.0]]), Y, -w, I, None,
                      r_min=0.05, with_visibility=False)
    r2 = float((Y * Y).sum())
    cos = y[2] / math.sqrt(r2)
    assert b[0] == pytest.approx((kd * I).sum() / math.pi * cos / max(r2, 0.05 ** 2), rel=1e-13)
    assert b[0] == pytest.approx(A.sum(), rel=1e-12)
