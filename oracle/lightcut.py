"""Global light cut (Sec. 3, step 1; Sec. 6, implementation of step 1).

TEST INFRASTRUCTURE ONLY (see the package header).

Step 1 of the method builds a light tree over every VPL and picks one cut of
it for the whole image with the lightcut method of Walter et al. (2005): a
node stays in the cut when the bound on the error of replacing its VPLs by
one representative light is small against the pixel's total, and is split
otherwise.  The paper states that the cut is error-bounded for the whole
image, that it is conservative because the visibility is over-estimated,
and (Sec. 6) that the split test runs for all nodes of one tree level at a
time.  It holds 800-900 nodes in the paper's scenes.

Readings (the paper defers the details to the lightcut paper):
* Tree.  The light tree over all VPLs (scenegen.full_light_tree): leaves are
  the VPLs perm[0 .. n), split node n + k has children left[k], right[k],
  every node's leaves are contiguous.  A node's light is built like the
  coarsening's node table (oracle.coarsen.node_table): the kept child is drawn
  by quantised intensity with Philox(key = (seed, 0),
  ctr = (node, 0, TAG_LTREE, 0)), I_f = fp32(fp64(I_l) + fp64(I_r)), the box
  is the union of the children's boxes.
* Error bound of node f at pixel x.  Every factor of an entry (Sec. 3's
  A(i, j), see oracle.shading) is bounded over the node's VPLs, the
  visibility by 1:
      bound(x, f) = G_ub * sum_c M_ub,c I_f,c,
      G_ub = c_ub / max(d_min^2, r_min^2),
      d_min = distance from x to f's box,
      c_ub = 0 if h <= 0, else min(1, h / d_min) (1 if d_min = 0),
      h = max over the box of n_x . (y - x) (taken at a corner),
      M_ub,c = kd_c / pi + ks (e + 2) / (2 pi) (the Phong lobe at its peak),
  the light-side cosine bounded by 1.  Both the node's true contribution and
  its representative's lie in [0, bound], so the bound holds for the error.
* Estimate of pixel x: the current cut's sum of unoccluded entries,
  est(x) = sum over cut nodes f and channels c of A_c(x, rep_f) with I_f and
  V = 1 (no shadow rays: the visibility is over-estimated here too).
* Whole image.  The test runs over a given set of sample pixels standing in
  for the image; f fails iff rho(f) = max over the samples of
  bound(x, f) / est(x) exceeds eps (b / 0 = inf for b > 0, 0 / 0 = 0; no
  samples: rho = 0).
* Level by level.  Level 0 is the root.  At each level every node of that
  level which is not a single VPL is tested against the estimate of the
  current cut; all failing nodes split at once and their children are the
  next level.  A node that passes stays in the cut and is not tested again.
* Cap.  A split adds one node to the cut.  When the failing nodes of a level
  would take the cut past max_cut, only the max_cut - |cut| of them with the
  largest rho split (ties to the lower node id), and the cut is final.
* Output.  The cut listed by smallest leaf (cluster k holds the VPLs
  perm[off[k] .. off[k+1])), and the tree above the cut in the coarsening's
  layout: the cut's nodes are leaves 0 .. n_g - 1 in cut order, the split
  nodes follow in increasing tree id (children before parents).

Ties.  A decision whose rho lies within AMBIG (relative) of eps, or a cap
choice between rhos within AMBIG of each other, is counted as ambiguous:
parity tests compare cuts only when the oracle reports none.

Pinned by: the bound's closed forms (a VPL on the normal facing the pixel,
Lambertian and Phong, and a VPL facing the pixel at any angle, Lambertian:
the bound equals the entry; a box below the horizon: 0), the bound against the brute-force sum over a node's VPLs on random
trees, the estimate of the all-leaves cut against the brute-force column sum
without occluders, a hand-worked four-VPL, two-pixel frame (rho of both
pairs and the cut for every eps and cap), and the cut's structure (a
partition of the VPLs, eps = 0 splits to single VPLs, the cap)
(tests/test_oracle_lightcut.py).
"""
from __future__ import annotations

import numpy as np

from .coarsen import node_table
from .shading import entries, point_arrays

TAG_LTREE = 8          # kept child of a split node of the full light tree
AMBIG = 1e-4
INV_PI = 1.0 / np.pi


def light_tree_table(vpls, perm, left, right, seed):
    """Node lights of the full light tree: leaf x is VPL perm[x]."""
    perm = np.asarray(perm, np.int64)
    pos = np.stack([vpls["x"], vpls["y"], vpls["z"]], axis=1).astype(np.float32)[perm]
    rgb = np.stack([vpls["ir"], vpls["ig"], vpls["ib"]], axis=1).astype(np.float32)[perm]
    return node_table(perm, rgb, pos, pos, np.ones(perm.shape[0], np.int64), left, right, seed, tag=TAG_LTREE)


def bound(x, nx, kd, ks, pe, lo, hi, inten, r_min):
    """Conservative error bound of nodes (boxes lo, hi, intensities inten)
    at pixels x (all arrays (E, 3) / (E,)), summed over the channels."""
    x = np.asarray(x, np.float64)
    nx = np.asarray(nx, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    gap = np.maximum(np.maximum(lo - x, x - hi), 0.0)
    d2 = np.einsum("ek,ek->e", gap, gap)
    d = np.sqrt(d2)
    h = np.maximum(nx * (lo - x), nx * (hi - x)).sum(axis=1)
    c_ub = np.where(h <= 0.0, 0.0, np.where(d > 0.0, np.minimum(1.0, h / np.where(d > 0.0, d, 1.0)), 1.0))
    g_ub = c_ub / np.maximum(d2, r_min * r_min)
    ks = np.asarray(ks, np.float64)
    pe = np.asarray(pe, np.float64)
    spec = np.where(ks > 0.0, ks * (pe + 2.0) * (0.5 * INV_PI), 0.0)
    m_ub = np.asarray(kd, np.float64) * INV_PI + spec[:, None]
    return g_ub * (m_ub * np.asarray(inten, np.float64)).sum(axis=1)


def _node_arrays(vpls, table, nodes):
    V = vpls
    rep = table["rep"][nodes]
    y = np.stack([V["x"], V["y"], V["z"]], axis=1).astype(np.float64)[rep]
    ny = np.stack([V["nx"], V["ny"], V["nz"]], axis=1).astype(np.float64)[rep]
    return y, ny, table["intensity"][nodes].astype(np.float64)


def estimate(points, sample_ids, vpls, table, cut, r_min):
    """est(x) for every sample pixel: unoccluded entries summed over the cut
    and the channels."""
    sample_ids = np.asarray(sample_ids, np.int64)
    cut = np.asarray(cut, np.int64)
    S, C = sample_ids.shape[0], cut.shape[0]
    est = np.zeros(S)
    if S == 0 or C == 0:
        return est
    y, ny, I = _node_arrays(vpls, table, cut)
    step = max(1, (1 << 20) // C)
    for a in range(0, S, step):
        b = min(S, a + step)
        ids = np.repeat(sample_ids[a:b], C)
        x, n, kd, ks, pe, wo = point_arrays(points, ids)
        A, _, _ = entries(x, n, kd, ks, pe, wo, np.tile(y, (b - a, 1)), np.tile(ny, (b - a, 1)),
                          np.tile(I, (b - a, 1)), None, r_min=r_min, with_visibility=False)
        est[a:b] = A.sum(axis=1).reshape(b - a, C).sum(axis=1)
    return est


def rho(points, sample_ids, table, nodes, est, r_min):
    """Worst ratio bound / est over the sample pixels for each node."""
    sample_ids = np.asarray(sample_ids, np.int64)
    nodes = np.asarray(nodes, np.int64)
    S, F = sample_ids.shape[0], nodes.shape[0]
    out = np.zeros(F)
    if S == 0 or F == 0:
        return out
    x, n, kd, ks, pe, _ = point_arrays(points, sample_ids)
    for k, f in enumerate(nodes):
        lo = np.repeat(table["lo"][f][None, :].astype(np.float64), S, axis=0)
        hi = np.repeat(table["hi"][f][None, :].astype(np.float64), S, axis=0)
        I = np.repeat(table["intensity"][f][None, :].astype(np.float64), S, axis=0)
        b = bound(x, n, kd, ks, pe, lo, hi, I, r_min)
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(est > 0.0, b / np.where(est > 0.0, est, 1.0), np.where(b > 0.0, np.inf, 0.0))
        out[k] = r.max()
    return out


def lightcut(points, vpls, perm, left, right, sample_ids, eps, max_cut, r_min=0.05, seed=0, table=None):
    """The global cut.  Returns a dict: cut (tree node ids by smallest leaf),
    offsets (n_cut + 1, into perm), above_left / above_right (the tree above
    the cut), rho (node -> tested ratio), levels (per level: tested, failing,
    split counts), ambiguous (count of near-tie decisions), table."""
    perm = np.asarray(perm, np.int64)
    n = perm.shape[0]
    assert n >= 1 and max_cut >= 1
    left = np.asarray(left, np.int64)
    right = np.asarray(right, np.int64)
    if table is None:
        table = light_tree_table(vpls, perm, left, right, seed)
    root = 2 * n - 2
    cut = [root]
    level = [root]
    tested = {}
    levels = []
    ambiguous = 0
    split_set = set()
    while level:
        inner = [f for f in level if f >= n]
        if not inner:
            break
        est = estimate(points, sample_ids, vpls, table, cut, r_min)
        r = rho(points, sample_ids, table, inner, est, r_min)
        for f, v in zip(inner, r):
            tested[f] = float(v)
            if np.isfinite(v) and abs(v - eps) <= AMBIG * eps:
                ambiguous += 1
        fail = [(float(v), f) for f, v in zip(inner, r) if v > eps]
        room = max_cut - len(cut)
        final = len(fail) > room
        if final:
            fail.sort(key=lambda t: (-t[0], t[1]))
            if 0 < room < len(fail):
                a, b = fail[room - 1][0], fail[room][0]     # a >= b; equal infinities go by id
                if np.isfinite(b) and a - b <= AMBIG * a:
                    ambiguous += 1
            fail = fail[:max(room, 0)]
        chosen = sorted(f for _, f in fail)
        levels.append(dict(tested=len(inner), failing=int((r > eps).sum()), split=len(chosen)))
        nxt = []
        cset = set(chosen)
        cut = [f for f in cut if f not in cset]
        for f in chosen:
            k = f - n
            cut += [int(left[k]), int(right[k])]
            nxt += [int(left[k]), int(right[k])]
            split_set.add(f)
        level = [] if final else nxt
    # cut by smallest leaf; tree above it in the coarsening layout
    min_leaf = table["min_leaf"]
    cut = sorted(cut, key=lambda f: int(min_leaf[f]))
    ng = len(cut)
    offsets = np.array([int(min_leaf[f]) for f in cut] + [n], np.int64)
    ids = {f: k for k, f in enumerate(cut)}
    split = sorted(split_set)
    for k, f in enumerate(split):
        ids[f] = ng + k
    above_left = np.array([ids[int(left[f - n])] for f in split], np.int64)
    above_right = np.array([ids[int(right[f - n])] for f in split], np.int64)
    return dict(cut=np.array(cut, np.int64), offsets=offsets, above_left=above_left, above_right=above_right,
                rho=tested, levels=levels, ambiguous=ambiguous, table=table)
