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
