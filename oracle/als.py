"""Per-row masked alternating least squares: a completion variant of the
slice matrix beside the paper's ADM (Appendix A).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper completes each slice with non-negative ADM; the classic
alternative for a matrix known only on Omega is masked ALS, where every row
of X (and every column of Y) is the exact least-squares fit to that row's
(column's) own observed entries.  With weighted regularisation (Zhou,
Wilkinson, Schreiber, Pan, "Large-scale parallel collaborative filtering for
the Netflix prize", 2008) the problem is

    min  sum_{(i,c) in Omega} (M_ic - x_i . y_c)^2
         + lam (sum_i n_i ||x_i||^2 + sum_c n_c ||y_c||^2),

n_i, n_c the observations in row i and column c, and one iteration solves,
for every row and then for every column,

    x_i = (sum_{c in Omega_i} y_c y_c^T + lam max(1, n_i) I)^-1 sum_{c in Omega_i} M_ic y_c
    y_c = (sum_{i in Omega^c} x_i x_i^T + lam max(1, n_c) I)^-1 sum_{i in Omega^c} M_ic x_i.

Readings shared with the ADM (so the two are compared on equal terms): the
stacked m' x 3n' matrix with a sample observing all three channels, the
scale s0 (M divided by its mean on Omega), the initial factors X0, Y0 (only
Y0 is used: the first half-step overwrites X), the relative residual on
Omega checked before each iteration, tol and the iteration cap.  Further
readings: lam = 0.01, fixed on the tiny workload (pixel RMSE against the full
VPL sum over 8 slices at 5% + 5%, 100 iterations: lam 0.001 0.174, 0.003
0.159, 0.01 0.154, 0.03 0.157, 0.05 0.162, 0.1 0.186, 0.3 0.297; the ADM
0.218); max(1, n) keeps a row or column without observations regular (its
factor becomes 0).  The 3 channels of a column j share its
rows (Omega^c is the same for c = j, n + j, 2n + j) but have their own y_c.

Pinned by: each half-step against the ridge least-squares fit of every row
solved by QR (numpy lstsq on [Y_obs^T; sqrt(lam n_i) I]), the objective
non-increasing over iterations, and recovery of a planted low-rank matrix
with a small lam (tests/test_oracle_als.py).
"""
import numpy as np
import scipy.linalg

LAM = 0.01


def residual(rows, cols, mvals, X, Y):
    return mvals - np.einsum("ek,ke->e", X[rows], Y[:, cols])


def half_step(rows, cols, mvals, n_out, F, lam):
    """The factor over `rows` (n_out x q) fitted to the fixed factor F
    (q x anything, indexed by `cols`): for each output index o, the ridge
    least-squares fit to its observations."""
    q = F.shape[0]
    out = np.zeros((n_out, q))
    order = np.argsort(rows, kind="stable")
    r, c, v = rows[order], cols[order], mvals[order]
    starts = np.searchsorted(r, np.arange(n_out + 1))
    for o in range(n_out):
        a, b = starts[o], starts[o + 1]
        Fo = F[:, c[a:b]]                                  # q x n_o
        G = Fo @ Fo.T + lam * max(1, b - a) * np.eye(q)
        out[o] = scipy.linalg.cho_solve(scipy.linalg.cho_factor(G, lower=True), Fo @ v[a:b])
    return out


def objective(rows, cols, mvals, m, N, X, Y, lam):
    R = residual(rows, cols, mvals, X, Y)
    ni = np.bincount(rows, minlength=m)
    nc = np.bincount(cols, minlength=N)
    return float(R @ R + lam * (np.maximum(1, ni) @ np.sum(X * X, axis=1)
                                + np.maximum(1, nc) @ np.sum(Y * Y, axis=0)))


def als(rows, cols, mvals, m, N, X0, Y0, lam, tol, max_iter, fixed_iters=False):
    """Masked ALS on the m x N matrix known at (rows, cols) = mvals.  Returns
    X (m x q), Y (q x N), iterations done, last relative residual on Omega."""
    X, Y = X0.copy(), Y0.copy()
    normM = float(np.sqrt(np.sum(mvals * mvals)))
    err = np.inf
    iters = max_iter
    for k in range(max_iter):
        Rv = residual(rows, cols, mvals, X, Y)
        err = float(np.sqrt(np.sum(Rv * Rv))) / normM if normM > 0 else 0.0
        if not fixed_iters and err < tol:
            iters = k
            break
        X = half_step(rows, cols, mvals, m, Y, lam)
        Y = half_step(cols, rows, mvals, N, X.T, lam).T
    return X, Y, iters, err
