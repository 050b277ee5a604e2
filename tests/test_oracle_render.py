"""Pins the oracle's frame pipeline, factorised column sum and brute force."""
import dataclasses
import math

import numpy as np

from oracle.render import Params, brute_force, reduce_factors, relative_rmse, render
from oracle.shading import entries, point_arrays
from scenegen import SceneConfig, make_scene

MICRO = SceneConfig("micro", 4, 4, 1.0, 2, 6, 6, 0.5, 16, "equal", n_slices=1)


def test_factorised_sum_identity():
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (7, 4))
    Y = rng.uniform(0, 1, (4, 15))
    I = reduce_factors(X, Y, 5, 2.5)
    Z = X @ Y
    expect = 2.5 * np.stack([Z[:, c * 5:(c + 1) * 5].sum(axis=1) for c in range(3)], axis=1)
    np.testing.assert_allclose(I, expect, rtol=1e-13)


def test_brute_force_is_the_exact_column_sum():
    sc = make_scene(MICRO, 3)
    p = Params()
    bf = brute_force(sc, p)
    V = sc.vpls
    for i in range(sc.m):
        x, n, kd, ks, pe, wo = point_arrays(sc.points, np.full(sc.n, i))
        pos = np.stack([V["x"], V["y"], V["z"]], axis=1).astype(np.float64)
        nrm = np.stack([V["nx"], V["ny"], V["nz"]], axis=1).astype(np.float64)
        inten = np.stack([V["ir"], V["ig"], V["ib"]], axis=1).astype(np.float64)
        A, _, _ = entries(x, n, kd, ks, pe, wo, pos, nrm, inten, sc.spheres)
        for c in range(3):
            assert abs(bf[i, c] - math.fsum(A[:, c])) <= 1e-14 * max(1.0, abs(bf[i, c]))
    # singleton cut: cluster sum equals the VPL sum exactly
    np.testing.assert_array_equal(brute_force(sc, p, mode="cut"), bf)


def test_full_sampling_pipeline_equals_brute_force():
    """100% sampling, singleton clusters, q = m': the method reproduces the
    brute-force image (the completed matrix equals M)."""
    sc = make_scene(MICRO, 5)
    assert sc.n_slices == 1 and sc.m == 16
    p = Params(pass1_ppm=500000, pass2_ppm=500000, max_iter=20000, tol=1e-13)
    I, per = render(sc, p)
    assert per[0]["N1"] + per[0]["N2"] == 16 * 6
    bf = brute_force(sc, p)
    np.testing.assert_allclose(I, bf, rtol=1e-7, atol=1e-9 * np.abs(bf).max())


def test_error_falls_as_rate_rises():
    sc = make_scene("tiny", 2)
    sl = [1, 9]
    pids = np.concatenate([sc.slice_rows(s) for s in sl])
    ref = brute_force(sc, Params(), point_ids=pids)
    errs = []
    for ppm in (20000, 100000):
        I, _ = render(sc, dataclasses.replace(Params(), pass1_ppm=ppm, pass2_ppm=ppm), slices=sl)
        errs.append(relative_rmse(I[pids], ref))
    assert errs[1] < errs[0]
