"""Non-negative completion of a sparsely sampled matrix by the alternating
direction method (Appendix A; the paper's solver after Xu, Yin, Wen, Zhang).

Problem: minimise ||P_Omega(X Y - M)||_F^2 over X >= 0 (m x q), Y >= 0
(q x N), rewritten with copies U = X, V = Y, U, V >= 0 and an auxiliary Z
with P_Omega(Z - M) = 0.  One iteration, in the appendix's order:

    X+ = (Z Y^T + alpha U - Lambda) (Y Y^T + alpha I)^-1
    Y+ = (X+^T X+ + beta I)^-1 (X+^T Z + beta V - Pi)
    Z+ = X+ Y+ + P_Omega(M - X+ Y+)
    U+ = P_+(X+ + Lambda / alpha),   V+ = P_+(Y+ + Pi / beta)
    Lambda+ = Lambda + gamma alpha (X+ - U+),   Pi+ = Pi + gamma beta (Y+ - V+)

Readings of the appendix's typos: the Y update multiplies X+^T Z (the
printed X+ Z^T has the wrong shape); the Lambda update adds to the old
Lambda; P_Omega KEEPS the entries in Omega and zeroes the rest (the
objective is restricted to the known entries and Z must equal M there);
X, Y >= 0 rather than > 0.

``adm`` runs the iteration in sparse-residual form, algebraically equal to
the dense one: with R = P_Omega(M - X Y) the Z of the current state is
X Y + R, hence Z Y^T = X (Y Y^T) + R Y^T and X+^T Z = (X+^T X) Y + X+^T R.
Only entries in Omega are ever touched.  ``adm_dense_step`` is the literal
dense transcription, kept to pin the sparse form.

Further readings (the paper gives no values): the stopping error is the
relative residual on Omega, ||R||_F / ||P_Omega M||_F, checked before each
update (stop when below tol or after max_iter updates); alpha = alpha0 N / q,
beta = beta0 m / q, gamma = 1.6; the initial factors are Philox draws
(``init_factors``) with E[(X0 Y0)_ij] = 1, M scaled to unit mean on Omega; U0 = X0,
V0 = Y0, Lambda0 = Pi0 = 0; Z0 = X0 Y0 + P_Omega(M - X0 Y0).

Non-negativity switch (a completion variant; the paper uses the
non-negative form): with nonneg off, U+ = X+ + Lambda / alpha and
V+ = Y+ + Pi / beta (no projection), so Lambda and Pi stay 0 and U = X+,
V = Y+: each half-step is then the proximal least-squares update
X+ = argmin ||Z - X Y||^2 + alpha ||X - X_k||^2.

Pinned by: the sparse form against the dense transcription, recovery of
planted non-negative rank-r matrices, exact data reproduction at 100%
sampling, and the KKT conditions at convergence; with nonneg off, one step
against the proximal least-squares problem solved by QR (numpy lstsq on the
stacked system [Y^T; sqrt(alpha) I]) and recovery of a planted matrix with
negative entries that the non-negative form cannot fit
(tests/test_oracle_adm.py, tests/test_oracle_als.py).
"""
import numpy as np
import scipy.linalg
import scipy.sparse

from .philox import TAG_INITX, TAG_INITY, philox4x64_vec, u24


def init_scale(q):
    return np.float32(2.0 / np.sqrt(float(q)))


def init_factors(seed, s, m, N, q):
    """X0 (m x q) and Y0 (q x N): fp32(u24(Philox(..)[0]) * fp32(2 / sqrt q)),
    counters (i, k, TAG_INITX, 0) and (k, col, TAG_INITY, 0), key (seed, s)."""
    cq = init_scale(q)
    ii, kk = np.meshgrid(np.arange(m, dtype=np.uint64), np.arange(q, dtype=np.uint64), indexing="ij")
    r = philox4x64_vec(seed, s, ii, kk, TAG_INITX, 0)[0]
    X0 = (u24(r).astype(np.float32) * cq).astype(np.float32)
    kk, cc = np.meshgrid(np.arange(q, dtype=np.uint64), np.arange(N, dtype=np.uint64), indexing="ij")
    r = philox4x64_vec(seed, s, kk, cc, TAG_INITY, 0)[0]
    Y0 = (u24(r).astype(np.float32) * cq).astype(np.float32)
    return X0.astype(np.float64), Y0.astype(np.float64)


def penalties(m, N, q, alpha0, beta0):
    return alpha0 * N / q, beta0 * m / q


def residual(rows, cols, mvals, X, Y):
    return mvals - np.einsum("ek,ke->e", X[rows], Y[:, cols])


def adm_step(rows, cols, mvals, m, N, X, Y, U, V, Lam, Pi, alpha, beta, gamma, Rv=None, nonneg=True):
    """One iteration in sparse-residual form; returns (X+, Y+, U+, V+, Lambda+, Pi+)."""
    q = X.shape[1]
    Iq = np.eye(q)
    if Rv is None:
        Rv = residual(rows, cols, mvals, X, Y)
    R = scipy.sparse.csr_matrix((Rv, (rows, cols)), shape=(m, N))
    GY = Y @ Y.T
    cY = scipy.linalg.cho_factor(GY + alpha * Iq, lower=True)
    rhsX = X @ GY + (R @ Y.T) + alpha * U - Lam               # = Z Y^T + alpha U - Lambda
    Xn = scipy.linalg.cho_solve(cY, rhsX.T).T                   # right-multiply by the inverse
    GX = Xn.T @ Xn
    cX = scipy.linalg.cho_factor(GX + beta * Iq, lower=True)
    rhsY = (Xn.T @ X) @ Y + np.asarray((R.T @ Xn).T) + beta * V - Pi   # = X+^T Z + beta V - Pi
    Yn = scipy.linalg.cho_solve(cX, rhsY)
    Un = Xn + Lam / alpha
    Vn = Yn + Pi / beta
    if nonneg:
        Un = np.maximum(0.0, Un)
        Vn = np.maximum(0.0, Vn)
    Lamn = Lam + gamma * alpha * (Xn - Un)
    Pin = Pi + gamma * beta * (Yn - Vn)
    return Xn, Yn, Un, Vn, Lamn, Pin


def adm(rows, cols, mvals, m, N, X0, Y0, alpha, beta, gamma, tol, max_iter, fixed_iters=False, nonneg=True):
    """Sparse-residual ADM.  rows/cols index the known entries of the
    m x N matrix, mvals their values.  Returns X, Y, iterations done, last
    relative residual, and the final (U, V, Lambda, Pi)."""
    X, Y = X0.copy(), Y0.copy()
    U, V = X0.copy(), Y0.copy()
    Lam = np.zeros_like(X)
    Pi = np.zeros_like(Y)
    normM = float(np.sqrt(np.sum(mvals * mvals)))
    err = np.inf
    iters = max_iter
    for k in range(max_iter):
        Rv = residual(rows, cols, mvals, X, Y)
        err = float(np.sqrt(np.sum(Rv * Rv))) / normM if normM > 0 else 0.0
        if not fixed_iters and err < tol:
            iters = k
            break
        X, Y, U, V, Lam, Pi = adm_step(rows, cols, mvals, m, N, X, Y, U, V, Lam, Pi,
                                       alpha, beta, gamma, Rv=Rv, nonneg=nonneg)
    return X, Y, iters, err, (U, V, Lam, Pi)


def adm_dense_step(M, mask, X, Y, U, V, Lam, Pi, Z, alpha, beta, gamma):
    """One iteration of the appendix written out on dense matrices."""
    q = X.shape[1]
    Iq = np.eye(q)
    Xn = (Z @ Y.T + alpha * U - Lam) @ np.linalg.inv(Y @ Y.T + alpha * Iq)
    Yn = np.linalg.inv(Xn.T @ Xn + beta * Iq) @ (Xn.T @ Z + beta * V - Pi)
    Zn = Xn @ Yn + mask * (M - Xn @ Yn)
    Un = np.maximum(0.0, Xn + Lam / alpha)
    Vn = np.maximum(0.0, Yn + Pi / beta)
    Lamn = Lam + gamma * alpha * (Xn - Un)
    Pin = Pi + gamma * beta * (Yn - Vn)
    return Xn, Yn, Zn, Un, Vn, Lamn, Pin
