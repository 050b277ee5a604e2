"""The seeded input generator produces well-formed inputs of the stated shapes."""
import numpy as np

import pytest

import scenegen
from scenegen import make_scene


def test_tiny_shapes_and_partitions():
    sc = make_scene("tiny", 1)
    assert sc.m == 4096 and sc.n == 1024 and sc.n_clusters == 1024 and sc.n_slices == 16
    assert np.all(np.diff(sc.pt_offsets) == 256)
    assert np.array_equal(np.sort(sc.pt_ids), np.arange(sc.m))
    assert np.array_equal(np.sort(sc.cut_members), np.arange(sc.n))
    assert np.all(sc.rank == 8)
    nrm = np.stack([sc.points["nx"], sc.points["ny"], sc.points["nz"]], 1).astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=1), 1.0, atol=1e-6)
    assert sc.vpls["z"].min() >= 0.25 and (sc.vpls["nz"] <= 0).all()
    top = (sc.spheres["cz"] + sc.spheres["r"]).max()
    assert top < 0.25


def test_deterministic():
    a = make_scene("tiny", 7)
    b = make_scene("tiny", 7)
    for k in a.points:
        assert np.array_equal(a.points[k], b.points[k])
    assert np.array_equal(a.pt_ids, b.pt_ids)


def test_cut_is_a_partition_for_clustered_config():
    from scenegen import CONFIGS
    import dataclasses
    cfg = dataclasses.replace(CONFIGS["mid"], width=64, height=64, n_slices=16, n_vpls=2048, n_clusters=256)
    sc = make_scene(cfg, 3)
    assert sc.n_clusters == 256
    assert np.array_equal(np.sort(sc.cut_members), np.arange(2048))
    assert np.all(np.diff(sc.cut_offsets) >= 1)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 301])
def test_full_light_tree_layout_and_node_sets(n):
    """Leaves contiguous under every node, children before parents, root last,
    and the same node sets the greedy cut sequence creates when grown to
    single VPLs."""
    rng = np.random.default_rng(n)
    pos = rng.uniform(size=(n, 3))
    perm, left, right = scenegen.full_light_tree(pos)
    assert sorted(perm.tolist()) == list(range(n))
    N = 2 * n - 1
    parent = -np.ones(N, np.int64)
    first = np.arange(N)
    last = np.arange(N)
    for k in range(n - 1):
        f, l, r = n + k, int(left[k]), int(right[k])
        assert l < f and r < f and parent[l] < 0 and parent[r] < 0
        parent[l] = parent[r] = f
        assert last[l] + 1 == first[r]
        first[f], last[f] = first[l], last[r]
    assert (parent[:N - 1] >= 0).all() and first[N - 1] == 0 and last[N - 1] == n - 1
    if n > 1:
        nodes, _, _ = scenegen.light_tree_cut_sequence(pos, rng.uniform(size=(n, 3)), n)
        assert {tuple(sorted(perm[first[f]:last[f] + 1])) for f in range(N)} == {tuple(x) for x in nodes}


def test_icosphere_is_a_closed_outward_mesh():
    from scenegen import icosphere
    for level in (0, 1, 2):
        V, F = icosphere(level)
        assert F.shape[0] == 20 * 4 ** level
        np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, rtol=1e-12)
        edges = {tuple(sorted(e)) for f in F for e in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0]))}
        assert V.shape[0] - len(edges) + F.shape[0] == 2          # Euler characteristic of a sphere
        n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
        assert (np.einsum("fk,fk->f", n, V[F].mean(axis=1)) > 0).all()   # every face wound outward


def test_triangle_scene_points_and_vpls_lie_on_faces():
    sc = make_scene("tri", 2)
    tri = sc.spheres["tri"].astype(np.float64).reshape(-1, 3, 3)
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    P = sc.points
    x = np.stack([P["px"], P["py"], P["pz"]], axis=1).astype(np.float64)
    nx = np.stack([P["nx"], P["ny"], P["nz"]], axis=1).astype(np.float64)

    def on_face(p, normal, lift):
        # some face whose plane is at distance `lift` along its normal and
        # whose projection contains the point, with the same normal
        d = np.einsum("tk,tk->t", n, p[None, :] - tri[:, 0])
        cand = np.nonzero((np.abs(d - lift) < 2e-5) & (np.einsum("tk,k->t", n, normal) > 1.0 - 1e-5))[0]
        for t in cand:
            q = p - lift * n[t]
            a, b, c = tri[t]
            w = np.linalg.lstsq(np.stack([b - a, c - a], axis=1), q - a, rcond=None)[0]
            if w.min() >= -1e-5 and w.sum() <= 1.0 + 1e-5:
                return True
        return False

    rng = np.random.default_rng(0)
    for i in rng.choice(sc.m, 200, replace=False):
        assert on_face(x[i], nx[i], 0.0), i
    V = sc.vpls
    y = np.stack([V["x"], V["y"], V["z"]], axis=1).astype(np.float64)
    ny = np.stack([V["nx"], V["ny"], V["nz"]], axis=1).astype(np.float64)
    for j in rng.choice(sc.n, 200, replace=False):
        assert on_face(y[j], ny[j], 2e-3), j
    # unit normals, every VPL inside the image region (paths leaving it are drawn again)
    np.testing.assert_allclose(np.linalg.norm(ny, axis=1), 1.0, rtol=1e-6)
    assert ((y[:, :2] >= 0.0) & (y[:, :2] <= 1.0)).all()
