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


def test_planted_low_rank_slice_below_full_sampling():
    """Below 100% sampling on a slice whose RGB matrix is exactly low rank
    and non-negative (A_c = U V_c^T, one U shared by the three channels):
    the first pass (uniform, 20%), the g weights from it and the second pass
    (20% more, Sec. 5), the completion of the stacked m x 3n matrix at q = 2
    (Appendix A) and the sum s0 X (Y e_c) (Sec. 3, step 5) give the exact
    column sums A_c e.  A wrong channel block, a dropped scale s0 or a sum
    over the wrong columns of Y fails it."""
    from oracle.render import complete_and_render, slice_weights
    from oracle.sampling import pass1, pass2

    rng = np.random.default_rng(12)
    m, n, q, seed, s = 48, 32, 2, 5, 3
    U = rng.uniform(0.2, 1.0, (m, q))
    V = rng.uniform(0.2, 1.0, (3, n, q)) * np.array([1.0, 0.5, 2.0])[:, None, None]
    A = np.einsum("ik,cjk->ijc", U, V)                              # (m, n, 3)
    i1, j1 = pass1(seed, s, m, n, 200000)
    w, _ = slice_weights(A[i1, j1], j1, n)
    taken = np.zeros(m * n, dtype=bool)
    taken[i1 * n + j1] = True
    i2, j2, short = pass2(seed, s, m, n, i1.shape[0], 200000, w, taken)
    assert not short and i1.shape[0] + i2.shape[0] == round(0.4 * m * n)
    ii, jj = np.concatenate([i1, i2]), np.concatenate([j1, j2])
    order = np.argsort(ii * n + jj, kind="stable")
    ii, jj = ii[order], jj[order]
    p = Params(seed=seed, max_iter=20000, tol=1e-12)
    I, iters, err, flags, _ = complete_and_render(m, n, q, ii, jj, A[ii, jj], seed, s, p)
    assert flags == 0 and err < 1e-11
    exact = A.sum(axis=1)                                            # (m, 3)
    np.testing.assert_allclose(I, exact, rtol=1e-6)
