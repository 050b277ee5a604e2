"""Pins the oracle's ADM completion (Appendix A)."""
import numpy as np

from oracle.adm import adm, adm_dense_step, adm_step, init_factors, init_scale, residual
from oracle.philox import TAG_INITX, TAG_INITY, philox4x64


def random_problem(m, N, q, frac, seed):
    rng = np.random.default_rng(seed)
    M = rng.uniform(0, 1, (m, N))
    mask = rng.uniform(0, 1, (m, N)) < frac
    rows, cols = np.nonzero(mask)
    return M, mask.astype(float), rows, cols, rng


def test_sparse_step_equals_dense_transcription():
    m, N, q = 9, 14, 4
    M, mask, rows, cols, rng = random_problem(m, N, q, 0.45, 1)
    X = rng.uniform(0, 1, (m, q))
    Y = rng.uniform(0, 1, (q, N))
    U = np.maximum(0, X + rng.normal(0, 0.1, X.shape))
    V = np.maximum(0, Y + rng.normal(0, 0.1, Y.shape))
    Lam = rng.normal(0, 0.2, X.shape)
    Pi = rng.normal(0, 0.2, Y.shape)
    alpha, beta, gamma = 0.7, 1.3, 1.6
    Z = X @ Y + mask * (M - X @ Y)
    d = adm_dense_step(M, mask, X, Y, U, V, Lam, Pi, Z, alpha, beta, gamma)
    s = adm_step(rows, cols, M[rows, cols], m, N, X, Y, U, V, Lam, Pi, alpha, beta, gamma)
    for a, b in zip((d[0], d[1], d[3], d[4], d[5], d[6]), s):
        np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-12)
    # and the Z of the next step is consistent: Z+ = X+Y+ + P(M - X+Y+)
    np.testing.assert_allclose(d[2][rows, cols], M[rows, cols], rtol=1e-14)


def test_planted_rank_r_recovery():
    rng = np.random.default_rng(7)
    m, N, r = 30, 40, 3
    Xs = rng.uniform(0, 1, (m, r))
    Ys = rng.uniform(0, 1, (r, N))
    M = Xs @ Ys
    mask = rng.uniform(0, 1, (m, N)) < 0.4
    rows, cols = np.nonzero(mask)
    X0, Y0 = init_factors(3, 0, m, N, r)
    X, Y, iters, err, _ = adm(rows, cols, M[rows, cols], m, N, X0, Y0, 0.1 * N / r, 0.1 * m / r,
                              1.6, 1e-12, 20000)
    assert err < 1e-10
    rel = np.linalg.norm(X @ Y - M) / np.linalg.norm(M)
    assert rel < 1e-6, rel


def test_full_sampling_reproduces_the_data():
    """100% sampling with q = m: the factorisation reproduces M, hence the
    factorised column sum X (Y e) equals the brute-force sum M e."""
    rng = np.random.default_rng(2)
    m, N = 8, 12
    M = rng.uniform(0, 1, (m, N)) * (rng.uniform(0, 1, (m, N)) > 0.3)
    rows, cols = np.nonzero(np.ones((m, N)))
    X0, Y0 = init_factors(5, 1, m, N, m)
    X, Y, iters, err, _ = adm(rows, cols, M[rows, cols], m, N, X0, Y0, 0.1 * N / m, 0.1, 1.6, 1e-13, 20000)
    e = np.ones(N)
    np.testing.assert_allclose(X @ (Y @ e), M @ e, rtol=1e-8, atol=1e-10)


def test_kkt_at_convergence():
    """ADM's fixed point satisfies the KKT conditions of the non-negative
    least-squares problem: X = U >= 0, Lambda = P(M - XY) Y^T (the negative
    gradient), Lambda = 0 where U > 0 and Lambda <= 0 where U = 0 (likewise
    Pi for Y).  ADM approaches it slowly, hence the loose bounds."""
    rng = np.random.default_rng(9)
    m, N, q = 12, 16, 3
    M = rng.uniform(0, 1, (m, N)) ** 3
    mask = rng.uniform(0, 1, (m, N)) < 0.6
    rows, cols = np.nonzero(mask)
    X0, Y0 = init_factors(2, 2, m, N, q)
    alpha, beta = 0.1 * N / q, 0.1 * m / q
    X, Y, iters, err, (U, V, Lam, Pi) = adm(rows, cols, M[rows, cols], m, N, X0, Y0, alpha, beta,
                                            1.6, 0.0, 10000, fixed_iters=True)
    assert np.abs(X - U).max() < 1e-5 and np.abs(Y - V).max() < 1e-5
    assert U.min() >= 0 and V.min() >= 0
    assert (U == 0).sum() > 0 and (V == 0).sum() > 0      # the bound is active somewhere
    R = np.zeros((m, N))
    R[rows, cols] = residual(rows, cols, M[rows, cols], X, Y)
    np.testing.assert_allclose(Lam, R @ Y.T, atol=1e-3)
    np.testing.assert_allclose(Pi, X.T @ R, atol=1e-3)
    pos = U > 1e-4
    assert np.abs(Lam[pos]).max() < 1e-3
    assert Lam[~pos].max(initial=-1.0) < 1e-3
    posv = V > 1e-4
    assert np.abs(Pi[posv]).max() < 1e-3
    assert Pi[~posv].max(initial=-1.0) < 1e-3


def test_init_factors_by_hand():
    q = 8
    X0, Y0 = init_factors(42, 3, 5, 7, q)
    cq = np.float32(2.0 / np.sqrt(8.0))
    assert init_scale(q) == cq
    r = philox4x64((42, 3), (4, 6, TAG_INITX, 0))[0]
    assert X0[4, 6] == float(np.float32(np.float32((r >> 40) / 2 ** 24) * cq))
    r = philox4x64((42, 3), (2, 5, TAG_INITY, 0))[0]
    assert Y0[2, 5] == float(np.float32(np.float32((r >> 40) / 2 ** 24) * cq))
    assert X0.min() >= 0 and X0.max() < cq and Y0.shape == (q, 7)


def test_tolerance_stops_early_and_fixed_iters_does_not():
    rng = np.random.default_rng(1)
    m, N, r = 10, 12, 2
    M = rng.uniform(0, 1, (m, r)) @ rng.uniform(0, 1, (r, N))
    rows, cols = np.nonzero(np.ones((m, N)))
    X0, Y0 = init_factors(1, 0, m, N, r)
    _, _, iters, err, _ = adm(rows, cols, M[rows, cols], m, N, X0, Y0, 0.5, 0.5, 1.6, 1e-3, 100)
    assert iters < 100 and err < 1e-3
    _, _, iters, _, _ = adm(rows, cols, M[rows, cols], m, N, X0, Y0, 0.5, 0.5, 1.6, 1e-3, 7, fixed_iters=True)
    assert iters == 7
