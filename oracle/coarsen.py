"""Per-slice light coarsening (Sec. 4) and the first pass it yields.

TEST INFRASTRUCTURE ONLY (see the package header).

The global cut's clusters are the leaves of a binary tree: the light tree's
nodes above the cut.  For each slice the coarsening repeatedly merges two
sibling nodes that are both in the slice's current cut, so the slice ends up
with a coarser cut of its own.

Sec. 4, as followed here:
* A merged node L_f keeps one child's light (L_f "is the same as L_a except
  intensity") and has intensity I_f = I_a + I_b.
* To judge a merge, pixels are drawn uniformly inside the slice, their number
  proportional to the light's intensity.  When both children were merged
  before, the pixel set is the union of theirs.
* The error of merging, over those pixels, is
  eps(L_f) = || V_b - V_a I_b / I_a ||_inf, with V_x the lighting of node x.
* The cost is cost(L_f) = eps(L_f) + cost(L_b), and cost is 0 for the
  leaves.
* Pairs are merged from the least cost on, until a target count of lights is
  reached or while the cost stays below an error bound.

Readings (the paper leaves these open):
* Representative.  The kept child a of split node f is drawn with probability
  proportional to the children's quantised total intensities,
  Q = max(1, floor(2^24 t / max(t_l, t_r))) with t = (R + G) + B in FP64 of
  the FP32 intensities.  The draw is a = left iff
  mulhi64(Philox(key = (seed, 0), ctr = (f, 0, TAG_TREE, 0))[0], Q_l + Q_r) < Q_l.
  I_f = fp32(fp64(I_l) + fp64(I_r)) per channel.
* Pixel sets.  Every leaf x of the global cut gets its own pixel set zeta_x:
  - its size is k_x = min(m', floor(K Q_x / sum Q)), with Q the same
    quantised intensities taken over all leaves and K the per-slice draw
    budget;
  - its members are the first k_x images of a keyed Feistel permutation of
    [0, m') with round function
    Philox(key = (seed, s), ctr = (R, r, TAG_ZETA, x))[0] & mask,
    cycle-walked into range.
  A node's pixel set is the union of its leaves' sets.  For two leaves this
  is a random set whose size is proportional to I_f; for two merged nodes it
  is the paper's zeta_a U zeta_b.  Repeated pixels do not change a max norm.
* The error.  With S_c(i, y) the per-channel lighting of pixel i by light y at
  unit intensity, V_x = S(., rep_x) * I_x, so
  V_b - V_a I_b / I_a = I_b * (S(., rep_b) - S(., rep_a)) channel by channel.
  eps is the max over the pixels and the three channels of that.  The form
  stays defined where I_a has a zero channel.
* Order and stop.  A pair becomes available once both children are leaves or
  merged nodes.  Available pairs are taken by the key
  (eff, height, node id), where eff(f) = max(cost(f), eff(children)) and
  eff(leaf) = 0.  So a pair that becomes available with a cost below the
  merge that freed it is taken next, and ties go to the lower node and then
  the lower id.  Merging continues while the slice has more than n_max
  columns, or while the least key's eff is below the bound.  It never goes
  below q columns (the slice's rank).
* Columns.  The coarsened cut's nodes are the slice's columns, ordered by the
  smallest leaf id below them.
* First pass (Sec. 5: the coarsening samples are the matrix samples).
  Omega1 = {(i, column of x) : x a leaf, i in zeta_x}.  Each pair is kept
  once; the list is in row-major order.

Pinned by: a hand-worked four-leaf tree (eps from closed-form entries, the
cost recursion, the merge order for every target count and a bound), the
heap order against a literal step-by-step scan of the available pairs on
random trees, the prefix-of-sorted-keys form the GPU computes, the pixel
sets' counts, distinctness and bijectivity, and the node table's sums and
draw frequencies (tests/test_oracle_coarsen.py).
"""
from __future__ import annotations

import dataclasses
import heapq

import numpy as np

from .philox import mulhi64, philox4x64, philox4x64_vec
from .shading import entries, point_arrays

TAG_TREE = 6    # kept child of a split node
TAG_ZETA = 7    # coarsening pixel draws
TWO24 = float(1 << 24)
FEISTEL_ROUNDS = 4


@dataclasses.dataclass
class CoarsenParams:
    pixels: int = 0          # K: draw budget of each slice over the leaves (sum of k_x <= K)
    bound: float = 0.0       # merge on while the least eff is below this (0: target count only)


def total_intensity(inten):
    """t = (R + G) + B in FP64 from FP32 intensities (n, 3)."""
    f = np.asarray(inten, np.float32).astype(np.float64)
    return (f[:, 0] + f[:, 1]) + f[:, 2]


def quantize(t):
    t = np.asarray(t, np.float64)
    tmax = t.max() if t.size else 0.0
    if not tmax > 0.0:
        return [1] * t.shape[0]
    return [int(max(1.0, np.floor(TWO24 * v / tmax))) for v in t]


def node_table(leaf_rep, leaf_int, leaf_lo, leaf_hi, leaf_members, left, right, seed, tag=TAG_TREE):
    """Every node of the tree above the cut: leaves 0 .. n_g - 1 (the cut's
    clusters), split nodes n_g .. 2 n_g - 2 (children first).  Returns a dict
    of arrays over the 2 n_g - 1 nodes.  ``tag`` keys the kept-child draws
    (the full light tree of the global cut uses its own)."""
    ng = int(np.asarray(leaf_rep).shape[0])
    N = 2 * ng - 1
    rep = np.zeros(N, np.int64)
    inten = np.zeros((N, 3), np.float32)
    kept = np.full(N, -1, np.int64)
    dropped = np.full(N, -1, np.int64)
    height = np.zeros(N, np.int64)
    parent = np.full(N, -1, np.int64)
    min_leaf = np.arange(N, dtype=np.int64)
    members = np.zeros(N, np.int64)
    lo = np.zeros((N, 3), np.float32)
    hi = np.zeros((N, 3), np.float32)
    rep[:ng] = leaf_rep
    inten[:ng] = leaf_int
    members[:ng] = leaf_members
    lo[:ng] = leaf_lo
    hi[:ng] = leaf_hi
    for k in range(ng - 1):
        f = ng + k
        l, r = int(left[k]), int(right[k])
        assert l < f and r < f and parent[l] < 0 and parent[r] < 0, "children must precede their parent once"
        parent[l] = parent[r] = f
        inten[f] = (inten[l].astype(np.float64) + inten[r].astype(np.float64)).astype(np.float32)
        ql, qr = quantize(total_intensity(inten[[l, r]]))
        u = mulhi64(philox4x64((seed, 0), (f, 0, tag, 0))[0], ql + qr)
        a, b = (l, r) if u < ql else (r, l)
        kept[f], dropped[f] = a, b
        rep[f] = rep[a]
        height[f] = 1 + max(height[l], height[r])
        min_leaf[f] = min(min_leaf[l], min_leaf[r])
        members[f] = members[l] + members[r]
        lo[f] = np.minimum(lo[l], lo[r])
        hi[f] = np.maximum(hi[l], hi[r])
    assert ng == 1 or (parent[:N - 1] >= 0).all(), "every node but the root has a parent"
    return dict(ng=ng, rep=rep, intensity=inten, kept=kept, dropped=dropped, height=height, parent=parent,
                min_leaf=min_leaf, members=members, lo=lo, hi=hi, left=np.asarray(left, np.int64),
                right=np.asarray(right, np.int64))


def node_lights(scene, table):
    """Light arrays of every node (representative position / normal, node
    intensity), in the layout oracle.render.eval_entries reads."""
    V = scene.vpls
    pos = np.stack([V["x"], V["y"], V["z"]], axis=1).astype(np.float64)[table["rep"]]
    nrm = np.stack([V["nx"], V["ny"], V["nz"]], axis=1).astype(np.float64)[table["rep"]]
    return dict(rep=table["rep"], intensity=table["intensity"], pos=pos, nrm=nrm, lo=table["lo"], hi=table["hi"])


def scene_table(scene, seed):
    from .cluster import cluster_table
    rep, inten, lo, hi = cluster_table(scene.vpls, scene.cut_offsets, scene.cut_members, seed)
    return node_table(rep, inten, lo, hi, np.diff(scene.cut_offsets), scene.tree_left, scene.tree_right, seed)


def leaf_quota(leaf_int, K):
    """k_x = floor(K Q_x / sum Q) in integers (before the cap at m')."""
    Q = quantize(total_intensity(leaf_int))
    tot = sum(Q)
    return np.array([(int(K) * q) // tot for q in Q], dtype=np.int64)


def _feistel(x, seed, s, h, word):
    x = np.asarray(x, dtype=np.uint64)
    mask = np.uint64((1 << h) - 1)
    L = x >> np.uint64(h)
    R = x & mask
    for rnd in range(FEISTEL_ROUNDS):
        F = philox4x64_vec(seed, s, R, rnd, TAG_ZETA, word)[0] & mask
        L, R = R, L ^ F
    return (L << np.uint64(h)) | R


def zeta_rows(seed, s, x, m, k):
    """The first k images of leaf x's keyed permutation of [0, m) (slice s)."""
    b = max(2, (int(m) - 1).bit_length())
    h = (b + 1) // 2
    out = _feistel(np.arange(k, dtype=np.uint64), seed, s, h, x)
    todo = np.nonzero(out >= np.uint64(m))[0]
    while todo.size:                     # cycle-walking
        out[todo] = _feistel(out[todo], seed, s, h, x)
        todo = todo[out[todo] >= np.uint64(m)]
    return out.astype(np.int64)


def greedy_merge(table, eps_of, n_max, bound, q, fp32=False):
    """The merge order of Sec. 4 over one slice.

    eps_of(f) -> eps of split node f.  Returns merged (list, in merge order),
    cost, eff (dicts over the nodes whose cost was computed).  With fp32 the
    cost sums are FP32 (as when the GPU's eps values decide)."""
    ng = table["ng"]
    left, right, dropped, parent, height = (table[k] for k in ("left", "right", "dropped", "parent", "height"))
    cost, eff = {}, {}
    merged = []
    done = np.zeros(2 * ng - 1, bool)
    done[:ng] = True
    heap = []

    def cost_of(x):
        return cost.get(x, 0.0) if x >= ng else 0.0

    def eff_of(x):
        return eff[x] if x >= ng else 0.0

    def make_available(f):
        e = eps_of(f)
        c = np.float32(np.float32(e) + np.float32(cost_of(int(dropped[f])))) if fp32 else e + cost_of(int(dropped[f]))
        k = f - ng
        cost[f] = float(c)
        eff[f] = max(float(c), eff_of(int(left[k])), eff_of(int(right[k])))
        heapq.heappush(heap, (eff[f], int(height[f]), f))

    for k in range(ng - 1):
        if left[k] < ng and right[k] < ng:
            make_available(ng + k)
    count = ng
    while heap and count > q:
        e, _, f = heap[0]
        if not (count > n_max or e < bound):
            break
        heapq.heappop(heap)
        merged.append(f)
        done[f] = True
        count -= 1
        p = int(parent[f])
        if p >= 0 and done[table["left"][p - ng]] and done[table["right"][p - ng]]:
            make_available(p)
    return merged, cost, eff


def final_columns(table, merged):
    """Nodes of the coarsened cut, ordered by their smallest leaf, and the
    column of every leaf."""
    ng = table["ng"]
    is_m = np.zeros(2 * ng - 1, bool)
    is_m[list(merged)] = True
    top = np.arange(ng)
    for x in range(ng):
        y = x
        while table["parent"][y] >= 0 and is_m[table["parent"][y]]:
            y = table["parent"][y]
        top[x] = y
    cols = np.unique(top)
    cols = cols[np.argsort(table["min_leaf"][cols], kind="stable")]
    col_of = {int(c): j for j, c in enumerate(cols)}
    return cols, np.array([col_of[int(t)] for t in top], np.int64)


def leaf_sets(table):
    """Leaves below every node (lists)."""
    ng = table["ng"]
    sets = [[x] for x in range(ng)]
    for k in range(ng - 1):
        sets.append(sets[table["left"][k]] + sets[table["right"][k]])
    return sets


def coarsen_slice(scene, table, s, seed, cp, n_max, params, eps_override=None):
    """Coarsen slice s.  Returns the coarsened cut (column node ids), Omega1
    (row-major (i, j)), the pixel sets, eps / cost / eff of the computed
    nodes, the merged nodes, the number of shadow-ray entries evaluated and
    whether any of them had an ambiguous visibility."""
    rows = scene.slice_rows(s)
    m = rows.shape[0]
    q = int(scene.rank[s])
    ng = table["ng"]
    k = np.minimum(leaf_quota(table["intensity"][:ng], cp.pixels), m)
    zeta = [zeta_rows(seed, s, x, m, int(k[x])) if k[x] > 0 else np.zeros(0, np.int64) for x in range(ng)]
    below = leaf_sets(table)
    L = node_lights(scene, table)
    eps_val, amb_nodes = {}, set()
    n_evals = [0]

    def eps_of(f):
        if eps_override is not None:
            eps_val[f] = float(eps_override[f])
            return eps_val[f]
        zr = np.concatenate([zeta[x] for x in below[f]]) if below[f] else np.zeros(0, np.int64)
        if zr.shape[0] == 0:
            eps_val[f] = 0.0
            return 0.0
        a, b = int(table["kept"][f]), int(table["dropped"][f])
        x, nn, kd, ks, pe, wo = point_arrays(scene.points, rows[zr])
        ones = np.ones((zr.shape[0], 3))
        Sa, amb_a, _ = entries(x, nn, kd, ks, pe, wo, np.repeat(L["pos"][[a]], zr.shape[0], 0),
                               np.repeat(L["nrm"][[a]], zr.shape[0], 0), ones, scene.spheres,
                               r_min=params.r_min, eps=params.ray_eps)
        Sb, amb_b, _ = entries(x, nn, kd, ks, pe, wo, np.repeat(L["pos"][[b]], zr.shape[0], 0),
                               np.repeat(L["nrm"][[b]], zr.shape[0], 0), ones, scene.spheres,
                               r_min=params.r_min, eps=params.ray_eps)
        n_evals[0] += 2 * zr.shape[0]
        if amb_a.any() or amb_b.any():
            amb_nodes.add(f)
        Ib = table["intensity"][b].astype(np.float64)
        eps_val[f] = float(np.max(Ib[None, :] * np.abs(Sb - Sa)))
        return eps_val[f]

    merged, cost, eff = greedy_merge(table, eps_of, n_max, cp.bound, q, fp32=eps_override is not None)
    cols, col_of_leaf = final_columns(table, merged)
    n = cols.shape[0]
    keys = set()
    for x in range(ng):
        for i in zeta[x]:
            keys.add(int(i) * n + int(col_of_leaf[x]))
    e = np.array(sorted(keys), np.int64)
    return dict(columns=cols, n=n, i1=e // n, j1=e % n, zeta=zeta, k=k, eps=eps_val, cost=cost, eff=eff,
                merged=merged, n_evals=n_evals[0], ambiguous_nodes=amb_nodes, col_of_leaf=col_of_leaf)


def render_slice_coarsened(scene, table, s, params, cp, n_max, weights_override=None, eps_override=None,
                           keep=False):
    """The whole method on slice s with coarsening (Sec. 3 steps 3-5): the
    coarsened cut, Omega1 from its pixel sets, g(j) and the second pass on the
    coarsened slice matrix, ADM, I(s) = X (Y e)."""
    from . import render as R
    from .sampling import pass2
    rows = scene.slice_rows(s)
    m = rows.shape[0]
    q = int(scene.rank[s])
    co = coarsen_slice(scene, table, s, params.seed, cp, n_max, params, eps_override=eps_override)
    L = node_lights(scene, table)
    n = co["n"]
    i1, j1 = co["i1"], co["j1"]
    A1, amb1, _ = R.eval_entries(scene, L, rows[i1], co["columns"][j1], params)
    w, st = R.slice_weights(A1, j1, n, params.pass2_mix)
    if weights_override is not None:
        w = np.asarray(weights_override, dtype=np.uint64)
    taken = np.zeros(m * n, dtype=bool)
    taken[i1 * n + j1] = True
    i2, j2, short = pass2(params.seed, s, m, n, i1.shape[0], params.pass2_ppm, w, taken)
    A2, amb2, _ = R.eval_entries(scene, L, rows[i2], co["columns"][j2], params)
    ii = np.concatenate([i1, i2])
    jj = np.concatenate([j1, j2])
    A = np.concatenate([A1, A2])
    order = np.argsort(ii * n + jj, kind="stable")
    ii, jj, A = ii[order], jj[order], A[order]
    I, iters, err, flags, fac = R.complete_and_render(m, n, q, ii, jj, A, params.seed, s, params)
    if short:
        flags |= R.FLAG_SHORTFALL
    out = dict(I=I, iters=iters, err=err, flags=flags, N1=int(i1.shape[0]), N2=int(i2.shape[0]), n=n,
               n_ambiguous=int(amb1.sum() + amb2.sum()), n_evals=co["n_evals"])
    if keep:
        out.update(co=co, i1=i1, j1=j1, A1=A1, w=w, stats=st, i2=i2, j2=j2, A2=A2, ii=ii, jj=jj, A=A,
                   amb1=amb1, amb2=amb2, factors=fac)
    return out


def render_coarsened(scene, params, cp, n_max, slices=None, weights_override=None, keep=False):
    """Radiance (m, 3) of the frame with per-slice coarsening; n_max: int or
    per-slice array of column caps."""
    table = scene_table(scene, params.seed)
    out = np.zeros((scene.m, 3))
    per = []
    caps = np.broadcast_to(np.asarray(n_max), (scene.n_slices,))
    for s in (range(scene.n_slices) if slices is None else slices):
        wo = None if weights_override is None else weights_override.get(s)
        r = render_slice_coarsened(scene, table, s, params, cp, int(caps[s]), weights_override=wo, keep=keep)
        out[scene.slice_rows(s)] = r["I"]
        per.append(r)
    return out, per
