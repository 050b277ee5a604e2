"""Pins of the completion variants in the oracle: masked ALS (oracle.als)
against an independent least-squares solve, its objective non-increasing, and
planted recovery; the ADM with non-negativity off (oracle.adm) against the
proximal least-squares step solved by QR, and recovery of a planted matrix
with negative entries that the non-negative form cannot fit."""
import numpy as np

from oracle import adm as A
from oracle import als as L


def sampled(m, N, frac, seed, signed=False, r=3):
    rng = np.random.default_rng(seed)
    if signed:
        M = rng.normal(size=(m, r)) @ rng.normal(size=(r, N))
    else:
        M = rng.uniform(0, 1, (m, r)) @ rng.uniform(0, 1, (r, N))
    k = int(frac * m * N)
    e = np.sort(rng.choice(m * N, k, replace=False))
    rows, cols = e // N, e % N
    return M, rows, cols, M[rows, cols]


def test_half_step_is_the_ridge_fit_of_every_row():
    m, N, q, lam = 12, 17, 4, 0.3
    M, rows, cols, v = sampled(m, N, 0.35, 1)
    F = np.random.default_rng(2).uniform(0, 1, (q, N))
    X = L.half_step(rows, cols, v, m, F, lam)
    for i in range(m):
        sel = rows == i
        n_i = int(sel.sum())
        Aug = np.vstack([F[:, cols[sel]].T, np.sqrt(lam * max(1, n_i)) * np.eye(q)])
        b = np.concatenate([v[sel], np.zeros(q)])
        want = np.linalg.lstsq(Aug, b, rcond=None)[0]
        assert np.allclose(X[i], want, rtol=1e-10, atol=1e-12), i
    # a row without observations gets 0
    X2 = L.half_step(rows[rows != 3], cols[rows != 3], v[rows != 3], m, F, lam)
    assert not X2[3].any()


def test_objective_never_increases():
    m, N, q, lam = 20, 30, 4, 0.05
    M, rows, cols, v = sampled(m, N, 0.3, 3)
    rng = np.random.default_rng(4)
    X, Y = rng.uniform(0, 1, (m, q)), rng.uniform(0, 1, (q, N))
    f = L.objective(rows, cols, v, m, N, X, Y, lam)
    for _ in range(15):
        X = L.half_step(rows, cols, v, m, Y, lam)
        f1 = L.objective(rows, cols, v, m, N, X, Y, lam)
        Y = L.half_step(cols, rows, v, N, X.T, lam).T
        f2 = L.objective(rows, cols, v, m, N, X, Y, lam)
        assert f1 <= f * (1 + 1e-12) and f2 <= f1 * (1 + 1e-12)
        f = f2


def test_masked_als_recovers_a_planted_low_rank_matrix():
    m, N, r = 40, 50, 3
    M, rows, cols, v = sampled(m, N, 0.4, 5, r=r)
    rng = np.random.default_rng(6)
    X0, Y0 = rng.uniform(0, 1, (m, r)), rng.uniform(0, 1, (r, N))
    X, Y, iters, err = L.als(rows, cols, v, m, N, X0, Y0, 1e-10, 1e-12, 3000)
    assert np.linalg.norm(X @ Y - M) / np.linalg.norm(M) < 1e-6


def test_adm_without_nonnegativity_is_a_proximal_least_squares_step():
    m, N, q = 15, 22, 3
    M, rows, cols, v = sampled(m, N, 0.4, 7)
    alpha, beta = A.penalties(m, N, q, 0.1, 0.1)
    rng = np.random.default_rng(8)
    X0, Y0 = rng.uniform(0, 1, (m, q)), rng.uniform(0, 1, (q, N))
    Lam, Pi = np.zeros((m, q)), np.zeros((q, N))
    Xn, Yn, Un, Vn, Lamn, Pin = A.adm_step(rows, cols, v, m, N, X0, Y0, X0.copy(), Y0.copy(), Lam, Pi,
                                          alpha, beta, 1.6, nonneg=False)
    Z = X0 @ Y0
    Z[rows, cols] = v
    Aug = np.vstack([Y0.T, np.sqrt(alpha) * np.eye(q)])
    want = np.linalg.lstsq(Aug, np.vstack([Z.T, np.sqrt(alpha) * X0.T]), rcond=None)[0].T
    assert np.allclose(Xn, want, rtol=1e-10, atol=1e-12)
    assert not Lamn.any() and not Pin.any()
    assert np.array_equal(Un, Xn) and np.array_equal(Vn, Yn)


def test_only_the_unconstrained_adm_fits_a_matrix_with_negative_entries():
    m, N, r = 30, 40, 2
    M, rows, cols, v = sampled(m, N, 0.5, 9, signed=True, r=r)
    rng = np.random.default_rng(10)
    X0, Y0 = rng.uniform(0, 1, (m, r)), rng.uniform(0, 1, (r, N))
    alpha, beta = A.penalties(m, N, r, 0.1, 0.1)
    errs = {}
    for nonneg in (True, False):
        X, Y, *_ = A.adm(rows, cols, v, m, N, X0, Y0, alpha, beta, 1.6, 1e-12, 4000, nonneg=nonneg)
        errs[nonneg] = np.linalg.norm(X @ Y - M) / np.linalg.norm(M)
    assert errs[False] < 1e-5 < 1e-2 < errs[True]


def test_render_by_either_completion():
    from oracle import render as R
    from scenegen import make_scene, scene_sample
    sc = scene_sample(make_scene("tiny", 2), [3])
    out = {}
    for method in ("adm", "als"):
        I, per = R.render(sc, R.Params(seed=2, max_iter=30, method=method))
        out[method] = I[sc.slice_rows(0)]
        assert np.isfinite(out[method]).all() and per[0]["iters"] <= 30
    ref = R.brute_force(sc, R.Params(seed=2), point_ids=sc.slice_rows(0))
    for method, I in out.items():
        assert R.relative_rmse(I, ref) < 0.5, method
