"""The SBVH over triangles (vplmc_sbvh_build, host only; Sec. 6 casts the
visibility rays through a spatial-split BVH): the layout the traversal relies
on (depth-first order, skip indices, contiguous leaf references), boxes that
contain their children and cover every part of every triangle (the
invariant spatial splits must keep), and a CPU walk of the same stackless
traversal that gives the brute-force visibility of the FP64 oracle."""
import numpy as np
import pytest

from oracle.shading import AMBIG_TRI, segment_triangle, triangle_visibility
from paper_2202_12567_amd import api
from scenegen import make_scene


@pytest.fixture(scope="module")
def tri_scene():
    sc = make_scene("tri", 1)
    tri = sc.spheres["tri"].astype(np.float64)
    box, code, refs = api.sbvh_build(sc.spheres["tri"])
    return sc, tri, box, code, refs


def test_layout(tri_scene):
    _, tri, box, code, refs = tri_scene
    n = box.shape[0]
    leaf, skip = code[:, 0], code[:, 1]
    assert n > 1 and skip[0] == n
    covered = np.zeros(refs.shape[0], np.int64)
    for k in range(n):
        assert k < skip[k] <= n
        if leaf[k] == 0:
            left, right = k + 1, skip[k + 1]
            assert right < skip[k] and skip[right] == skip[k]      # two children exactly span the subtree
            for c in (left, right):
                assert (box[c, :3] >= box[k, :3]).all() and (box[c, 3:] <= box[k, 3:]).all()
        else:
            first, cnt = leaf[k] >> 4, leaf[k] & 15
            assert 1 <= cnt <= 15 and skip[k] == k + 1
            covered[first:first + cnt] += 1
    assert (covered == 1).all()                    # leaf references are contiguous and disjoint
    assert np.array_equal(np.unique(refs), np.arange(tri.shape[0]))   # every triangle is referenced


def test_every_part_of_every_triangle_is_in_a_leaf_box(tri_scene):
    _, tri, box, code, refs = tri_scene
    leaf = code[:, 0]
    leaves = np.nonzero(leaf)[0]
    owner = [[] for _ in range(tri.shape[0])]
    for k in leaves:
        first, cnt = leaf[k] >> 4, leaf[k] & 15
        for r in refs[first:first + cnt]:
            owner[r].append(k)
    rng = np.random.default_rng(0)
    for t in range(tri.shape[0]):
        a, b, c = tri[t, 0:3], tri[t, 3:6], tri[t, 6:9]
        u = rng.uniform(0.0, 1.0, (16, 2))
        u = np.where(u.sum(axis=1, keepdims=True) > 1.0, 1.0 - u, u)
        pts = np.concatenate([np.stack([a, b, c]), a + u[:, :1] * (b - a) + u[:, 1:] * (c - a)])
        bx = box[owner[t]].astype(np.float64)
        inside = ((pts[:, None, :] >= bx[None, :, :3]) & (pts[:, None, :] <= bx[None, :, 3:])).all(axis=2)
        assert inside.any(axis=1).all(), f"triangle {t}: a point lies in none of its leaves' boxes"


def _walk(o, D, box, code, refs, tri):
    """The device traversal on the CPU: slab test in FP64, left child on an
    inner hit, else the skip index; a leaf tests its references."""
    leaf, skip = code[:, 0], code[:, 1]
    n = box.shape[0]
    inv = 1.0 / np.where(np.abs(D) > 1e-20, D, np.copysign(1e-20, D))
    node = 0
    while node < n:
        t0 = (box[node, :3] - o) * inv
        t1 = (box[node, 3:] - o) * inv
        tmin = max(np.minimum(t0, t1).max(), 0.0)
        tmax = min(np.maximum(t0, t1).min(), 1.0)
        hit = tmin <= tmax
        if hit and leaf[node] != 0:
            first, cnt = leaf[node] >> 4, leaf[node] & 15
            tr = tri[refs[first:first + cnt]]
            m, _ = segment_triangle(o[None], D[None], tr[:, 0:3], tr[:, 3:6], tr[:, 6:9])
            if (m > 0.0).any():
                return 0.0
        node = node + 1 if (hit and leaf[node] == 0) else skip[node]
    return 1.0


def test_traversal_matches_brute_force(tri_scene):
    sc, tri, box, code, refs = tri_scene
    rng = np.random.default_rng(5)
    P = sc.points
    ids = rng.integers(0, sc.m, 400)
    vs = rng.integers(0, sc.n, 400)
    x = np.stack([P["px"][ids], P["py"][ids], P["pz"][ids]], axis=1).astype(np.float64)
    nx = np.stack([P["nx"][ids], P["ny"][ids], P["nz"][ids]], axis=1).astype(np.float64)
    y = np.stack([sc.vpls["x"][vs], sc.vpls["y"][vs], sc.vpls["z"][vs]], axis=1).astype(np.float64)
    o = x + 1e-4 * nx
    V, amb = triangle_visibility(o, y, tri)
    blocked = 0
    for k in range(o.shape[0]):
        if amb[k]:
            continue
        assert _walk(o[k], y[k] - o[k], box.astype(np.float64), code, refs, tri) == V[k], k
        blocked += V[k] == 0.0
    assert 20 < blocked < 380


def test_spatial_splits_chop_long_triangles():
    # two long slivers crossing a cloud of small triangles: the slivers are
    # referenced from several leaves (spatial splits), each small one once
    rng = np.random.default_rng(3)
    c = rng.uniform(0.0, 1.0, (300, 3))
    small = np.concatenate([c, c + [0.01, 0, 0], c + [0, 0.01, 0]], axis=1)
    long_ = np.array([[0.0, 0.5, 0.5, 1.0, 0.5, 0.5, 1.0, 0.51, 0.5],
                      [0.5, 0.0, 0.5, 0.5, 1.0, 0.5, 0.51, 1.0, 0.5]])
    tri = np.concatenate([small, long_]).astype(np.float32)
    _, _, refs = api.sbvh_build(tri)
    counts = np.bincount(refs, minlength=tri.shape[0])
    assert (counts[:300] >= 1).all() and (counts[300:] >= 2).all()


def test_rejects_bad_input():
    lib = api.N.load()
    import ctypes
    nn, nr = ctypes.c_int32(), ctypes.c_int32()
    bad = np.zeros(9, np.float32)
    bad[4] = np.nan
    assert lib.vplmc_sbvh_build(1, bad.ctypes.data_as(ctypes.c_void_p), 0, None, None, 0, None,
                                ctypes.byref(nn), ctypes.byref(nr)) == api.N.EINVAL
    assert lib.vplmc_sbvh_build(-1, None, 0, None, None, 0, None, ctypes.byref(nn), ctypes.byref(nr)) == api.N.EINVAL
    # room for too few nodes: an error, counts still reported
    tri = np.random.default_rng(1).uniform(0, 1, (50, 9)).astype(np.float32)
    assert lib.vplmc_sbvh_build(50, tri.ctypes.data_as(ctypes.c_void_p), 1, None, None, 1000, None,
                                ctypes.byref(nn), ctypes.byref(nr)) == api.N.EINVAL and nn.value > 1


def test_duplication_budget():
    # a grid of long slivers crossing each other everywhere: spatial splits
    # would chop them without end; the references stay within twice the
    # triangles and the structure stays valid
    k = 60
    t = np.linspace(0.0, 1.0, k)
    xs = [[0.0, y, 0.0, 1.0, y, 0.0, 1.0, y + 1e-3, 0.0] for y in t]
    ys = [[x, 0.0, 0.01, x, 1.0, 0.01, x + 1e-3, 1.0, 0.01] for x in t]
    tri = np.array(xs + ys, np.float32)
    box, code, refs = api.sbvh_build(tri)
    assert refs.shape[0] <= 2 * tri.shape[0]
    assert np.array_equal(np.unique(refs), np.arange(tri.shape[0]))
    assert code[0, 1] == box.shape[0]
