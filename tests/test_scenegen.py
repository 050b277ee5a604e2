"""The seeded input generator produces well-formed inputs of the stated shapes."""
import numpy as np

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
