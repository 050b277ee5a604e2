"""The whole method on one frame, slice by slice, and the brute-force image it
approximates.

Image (Sec. 3): the rendered image is the sum of the columns of the
lighting matrix, I_i = sum_j A(i, j).  ``brute_force`` computes that sum
over every VPL (the paper's reference images, Sec. 6, Fig. 2) or over the
clusters of a cut.

Per slice (Sec. 3 steps 4-5, Sec. 5, Appendix A):
  a0 cluster table (rep, intensity)                         -> oracle.cluster
  a1 first pass, uniform distinct entries                   -> oracle.sampling.pass1
  a2 entries at the samples                                 -> oracle.shading
  a3 g(j) = max - min over the first pass, integer weights  -> oracle.sampling
  a5 second pass by g                                        -> oracle.sampling.pass2
  a7 ADM completion of the stacked m' x 3n' matrix
     [M_R | M_G | M_B] (one shared X; reading: all three channels of an
     entry are observed together) after scaling by the mean
     observed value s0 = sum M / (3 |Omega|), so that the initial
     E[(X0 Y0)_ij] = 1 predicts the observed mean       -> oracle.adm
  a8 I(s) = s0 X (Y e), per channel                          (Sec. 3, step 5)

Pinned by: brute force against math.fsum entry by entry; at 100% sampling
with singleton clusters and q = min(m', 3n') the pipeline reproduces the
brute-force sum; X (Y e) = (X Y) e; at 40% sampling (both passes, g
weights) a slice matrix that is exactly non-negative and of rank q is
completed and summed to its exact column sums (tests/test_oracle_render.py).
The whole method below 100% sampling on rendered scenes has no worked
example in the paper: parity unpinned against the paper for that case
(pinned only by the stage pins above, the planted low-rank slice and the
trend that the error falls as the rate rises, Sec. 6).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import adm as adm_mod
from .cluster import cluster_table
from .sampling import column_stats, count_from_ppm, importance, pass1, pass2, weights_from_g
from .shading import entries, point_arrays

FLAG_ALL_ZERO = 1
FLAG_NOT_CONVERGED = 2
FLAG_SHORTFALL = 4


@dataclasses.dataclass
class Params:
    seed: int = 1
    pass1_ppm: int = 50000
    pass2_ppm: int = 50000
    max_iter: int = 100
    tol: float = 1e-3
    alpha0: float = 0.1
    beta0: float = 0.1
    gamma: float = 1.6
    r_min: float = 0.05
    # completion: "adm" (Appendix A) or "als" (per-row masked ALS, oracle.als);
    # nonneg False switches the ADM's projection off; lam the ALS regulariser
    method: str = "adm"
    nonneg: bool = True
    lam: float = 0.01
    ray_eps: float = 1e-4
    fixed_iters: bool = False
    # second-pass density g(j) + pass2_mix mean g (0: the paper's g; inf: uniform)
    pass2_mix: float = 0.0


def cluster_lights(scene, seed):
    rep, inten, lo, hi = cluster_table(scene.vpls, scene.cut_offsets, scene.cut_members, seed)
    V = scene.vpls
    pos = np.stack([V["x"], V["y"], V["z"]], axis=1).astype(np.float64)[rep]
    nrm = np.stack([V["nx"], V["ny"], V["nz"]], axis=1).astype(np.float64)[rep]
    return dict(rep=rep, intensity=inten, pos=pos, nrm=nrm, lo=lo, hi=hi)


def eval_entries(scene, lights, rows, cols, params):
    """Entries A(rows[k], cols[k]) for global point ids / cluster ids."""
    x, n, kd, ks, pe, wo = point_arrays(scene.points, rows)
    A, amb, lit = entries(x, n, kd, ks, pe, wo, lights["pos"][cols], lights["nrm"][cols],
                          lights["intensity"][cols].astype(np.float64), scene.spheres,
                          r_min=params.r_min, eps=params.ray_eps)
    return A, amb, lit


def slice_first_pass(scene, lights, s, params):
    rows = scene.slice_rows(s)
    cols = scene.slice_cols(s)
    m, n = rows.shape[0], cols.shape[0]
    i1, j1 = pass1(params.seed, s, m, n, params.pass1_ppm)
    A1, amb1, lit1 = eval_entries(scene, lights, rows[i1], cols[j1], params)
    return i1, j1, A1, amb1, lit1


def slice_weights(A1, j1, n, mix=0.0):
    t = A1.sum(axis=1)
    cnt, mean, var, mn, mx = column_stats(j1, t, n)
    g = importance(mn, mx, cnt)
    return weights_from_g(g, mix), dict(count=cnt, mean=mean, var=var, min=mn, max=mx, g=g)


def complete_and_render(m, n, q, ii, jj, A, seed, s, params, X0Y0=None):
    """ADM on the stacked m x 3n matrix from entries (ii, jj, RGB A); returns
    per-point RGB radiance of the slice, iterations, residual, flags."""
    flags = 0
    nOmega = ii.shape[0]
    sumsq = float(np.sum(A * A))
    if nOmega == 0 or not sumsq > 0.0:
        return np.zeros((m, 3)), 0, 0.0, FLAG_ALL_ZERO, None
    s0 = float(np.sum(A)) / (3.0 * nOmega)
    N = 3 * n
    rows = np.concatenate([ii, ii, ii])
    cols = np.concatenate([jj, jj + n, jj + 2 * n])
    mvals = np.concatenate([A[:, 0], A[:, 1], A[:, 2]]) / s0
    if X0Y0 is None:
        X0, Y0 = adm_mod.init_factors(params.seed, s, m, N, q)
    else:
        X0, Y0 = X0Y0
    if params.method == "als":
        from . import als as als_mod
        X, Y, iters, err = als_mod.als(rows, cols, mvals, m, N, X0, Y0, params.lam, params.tol, params.max_iter,
                                       params.fixed_iters)
    else:
        alpha, beta = adm_mod.penalties(m, N, q, params.alpha0, params.beta0)
        X, Y, iters, err, _ = adm_mod.adm(rows, cols, mvals, m, N, X0, Y0, alpha, beta, params.gamma,
                                          params.tol, params.max_iter, params.fixed_iters, nonneg=params.nonneg)
    if iters >= params.max_iter and not params.fixed_iters:
        flags |= FLAG_NOT_CONVERGED
    I = reduce_factors(X, Y, n, s0)
    return I, iters, err, flags, (X, Y, s0)


def reduce_factors(X, Y, n, s0):
    """I^c = s0 X (Y e_c): e_c sums the n columns of channel c (Sec. 3, step 5)."""
    w = np.stack([Y[:, c * n:(c + 1) * n].sum(axis=1) for c in range(3)], axis=1)   # q x 3
    return s0 * (X @ w)


def render_slice(scene, lights, s, params, weights_override=None, keep=False):
    rows = scene.slice_rows(s)
    cols = scene.slice_cols(s)
    m, n = rows.shape[0], cols.shape[0]
    q = int(scene.rank[s])
    D = m * n
    i1, j1, A1, amb1, _ = slice_first_pass(scene, lights, s, params)
    w, st = slice_weights(A1, j1, n, params.pass2_mix)
    if weights_override is not None:
        w = np.asarray(weights_override, dtype=np.uint64)
    taken = np.zeros(D, dtype=bool)
    taken[i1 * n + j1] = True
    N1 = i1.shape[0]
    i2, j2, short = pass2(params.seed, s, m, n, N1, params.pass2_ppm, w, taken)
    A2, amb2, _ = eval_entries(scene, lights, rows[i2], cols[j2], params)
    ii = np.concatenate([i1, i2])
    jj = np.concatenate([j1, j2])
    A = np.concatenate([A1, A2])
    order = np.argsort(ii * n + jj, kind="stable")        # CSR (row-major) order
    ii, jj, A = ii[order], jj[order], A[order]
    I, iters, err, flags, fac = complete_and_render(m, n, q, ii, jj, A, params.seed, s, params)
    if short:
        flags |= FLAG_SHORTFALL
    out = dict(I=I, iters=iters, err=err, flags=flags, N1=N1, N2=int(i2.shape[0]),
               n_ambiguous=int(amb1.sum() + amb2.sum()))
    if keep:
        out.update(i1=i1, j1=j1, A1=A1, w=w, stats=st, i2=i2, j2=j2, A2=A2, ii=ii, jj=jj, A=A,
                   amb1=amb1, amb2=amb2, factors=fac)
    return out


def render(scene, params, slices=None, weights_override=None, keep=False):
    """Radiance (m, 3) FP64 of the frame (points outside the slices stay 0)."""
    lights = cluster_lights(scene, params.seed)
    out = np.zeros((scene.m, 3))
    per = []
    for s in (range(scene.n_slices) if slices is None else slices):
        wo = None if weights_override is None else weights_override.get(s)
        r = render_slice(scene, lights, s, params, weights_override=wo, keep=keep)
        out[scene.slice_rows(s)] = r["I"]
        per.append(r)
    return out, per


def brute_force(scene, params, mode="vpls", point_ids=None, chunk=1 << 20):
    """Column sum of the full lighting matrix: every VPL (mode "vpls") or
    every cluster of the cut (mode "cut"), FP64 entries and sums."""
    if mode == "vpls":
        V = scene.vpls
        pos = np.stack([V["x"], V["y"], V["z"]], axis=1).astype(np.float64)
        nrm = np.stack([V["nx"], V["ny"], V["nz"]], axis=1).astype(np.float64)
        inten = np.stack([V["ir"], V["ig"], V["ib"]], axis=1).astype(np.float64)
    else:
        L = cluster_lights(scene, params.seed)
        pos, nrm, inten = L["pos"], L["nrm"], L["intensity"].astype(np.float64)
    pids = np.arange(scene.m) if point_ids is None else np.asarray(point_ids)
    nl = pos.shape[0]
    out = np.zeros((pids.shape[0], 3))
    rows_per = max(1, chunk // nl)
    for a in range(0, pids.shape[0], rows_per):
        b = min(pids.shape[0], a + rows_per)
        pr = np.repeat(pids[a:b], nl)
        lj = np.tile(np.arange(nl), b - a)
        x, n, kd, ks, pe, wo = point_arrays(scene.points, pr)
        A, _, _ = entries(x, n, kd, ks, pe, wo, pos[lj], nrm[lj], inten[lj], scene.spheres,
                          r_min=params.r_min, eps=params.ray_eps)
        out[a:b] = A.reshape(b - a, nl, 3).sum(axis=1)
    return out


def relative_rmse(I, ref):
    ref = np.asarray(ref, np.float64)
    d = np.asarray(I, np.float64) - ref
    return float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(ref * ref)))


__all__ = ["Params", "render", "render_slice", "brute_force", "relative_rmse", "cluster_lights",
           "complete_and_render", "reduce_factors", "count_from_ppm"]
