"""The sphere BVH (vplmc_bvh_build, host only): the layout the stackless
traversal relies on (depth-first order, every skip index past its node, the
left child right after its parent, the two children exactly spanning the
subtree), every sphere in exactly one leaf, every box containing its
children and its spheres (padded), and a CPU walk of the traversal giving
the oracle's brute-force visibility on scene segments: the tree's shape
decides which boxes a ray visits, never its answer."""
import numpy as np
import pytest

from oracle.shading import segment_sphere_dist, visibility
from paper_2202_12567_amd import api
from scenegen import make_scene


@pytest.fixture(scope="module", params=["tiny", "mid"])
def built(request):
    sc = make_scene(request.param, 3)
    box, code, order = api.bvh_build(sc.spheres)
    return sc, box, code, order


def test_layout_and_membership(built):
    sc, box, code, order = built
    n = box.shape[0]
    leaf, skip = code[:, 0], code[:, 1]
    S = sc.spheres["r"].shape[0]
    assert np.array_equal(np.sort(order), np.arange(S))
    seen = np.zeros(S, np.int64)
    c = np.stack([sc.spheres["cx"], sc.spheres["cy"], sc.spheres["cz"]], axis=1).astype(np.float64)
    r = sc.spheres["r"].astype(np.float64)
    assert skip[0] == n
    for k in range(n):
        assert k < skip[k] <= n
        if leaf[k] == 0:
            left, right = k + 1, skip[k + 1]
            assert right < skip[k] and skip[right] == skip[k]
            for ch in (left, right):
                assert (box[ch, :3] >= box[k, :3]).all() and (box[ch, 3:] <= box[k, 3:]).all()
        else:
            first, cnt = leaf[k] >> 4, leaf[k] & 15
            assert 1 <= cnt <= 4 and skip[k] == k + 1
            ids = order[first:first + cnt]
            seen[ids] += 1
            assert ((c[ids] - r[ids, None]) > box[k, :3]).all() and ((c[ids] + r[ids, None]) < box[k, 3:]).all()
    assert (seen == 1).all()


def _walk(o, D, box, code, order, c, r):
    leaf, skip = code[:, 0], code[:, 1]
    n = box.shape[0]
    inv = 1.0 / np.where(np.abs(D) > 1e-20, D, np.copysign(1e-20, D))
    node = 0
    while node < n:
        t0 = (box[node, :3] - o) * inv
        t1 = (box[node, 3:] - o) * inv
        hit = max(np.minimum(t0, t1).max(), 0.0) <= min(np.maximum(t0, t1).min(), 1.0)
        if hit and leaf[node] != 0:
            ids = order[(leaf[node] >> 4):(leaf[node] >> 4) + (leaf[node] & 15)]
            if (segment_sphere_dist(o[None], D[None], c[ids])[0] < r[ids]).any():
                return 0.0
        node = node + 1 if (hit and leaf[node] == 0) else skip[node]
    return 1.0


def test_traversal_matches_brute_force(built):
    sc, box, code, order = built
    c = np.stack([sc.spheres["cx"], sc.spheres["cy"], sc.spheres["cz"]], axis=1).astype(np.float64)
    r = sc.spheres["r"].astype(np.float64)
    rng = np.random.default_rng(6)
    P = sc.points
    ids = rng.integers(0, sc.m, 300)
    vs = rng.integers(0, sc.n, 300)
    x = np.stack([P["px"][ids], P["py"][ids], P["pz"][ids]], axis=1).astype(np.float64)
    nx = np.stack([P["nx"][ids], P["ny"][ids], P["nz"][ids]], axis=1).astype(np.float64)
    y = np.stack([sc.vpls["x"][vs], sc.vpls["y"][vs], sc.vpls["z"][vs]], axis=1).astype(np.float64)
    o = x + 1e-4 * nx
    V, amb = visibility(o, y, sc.spheres)
    for k in range(o.shape[0]):
        if not amb[k]:
            assert _walk(o[k], y[k] - o[k], box.astype(np.float64), code, order, c, r) == V[k], k
    assert 10 < (V == 0).sum() < 290


def test_rejects_bad_spheres():
    import ctypes
    lib = api.N.load()
    nn = ctypes.c_int32()
    a = np.zeros(1, np.float32)
    bad_r = np.zeros(1, np.float32)
    f = lambda v: v.ctypes.data_as(ctypes.c_void_p)
    assert lib.vplmc_bvh_build(1, f(a), f(a), f(a), f(bad_r), 10, None, None, None, ctypes.byref(nn)) == api.N.EINVAL
