"""Seeded synthetic scenes shaped like the paper's many-light workloads.

This module is the one piece of code that both the product path's callers
(tests, benchmark) and the FP64 oracle read: it draws the INPUTS of the
method -- surface points seen by a camera, VPLs, occluder spheres, a light
tree cut, and the slices -- and holds none of the method's arithmetic (no
shading, no sampling, no completion, no cluster representative or
intensity).  Everything is seeded with ``numpy.random.default_rng(seed)``.

Recipe (stands in for the paper's Bedroom/Tearoom/Museum scenes, which are
not available; Sec. 6, Table 1 gives their shapes: 480K-786K pixels,
50K-231K VPLs, a few hundred cut nodes per slice, ~800-pixel slices):

* camera: orthographic, looking down -z; pixel (u, v) shoots a ray from
  z = 10 over [0, W_r] x [0, 1]; the nearest hit on the plane z = 0 or on a
  sphere is the surface point, its normal comes from the geometry, and the
  viewer direction is +z;
* spheres rest on the plane (centre z = radius), centres uniform over the
  region, radius U[0.02, 0.1];
* materials per object (plane = object 0): albedo U[0.2, 0.9]^3; an object
  is Phong with probability ``phong_prob`` (diffuse 0.75 * albedo, specular
  0.2 white, exponent U[10, 100]), else Lambertian;
* VPLs: position U[region] x U[0.25, 1.0] (always above every sphere),
  normal = minus a cosine-weighted direction about +z, RGB U[0, 1]^3;
* light tree: median split along the longest bbox axis; the cut grows by
  splitting the node with the largest (sum RGB) * (bbox diagonal), ties to
  the lower node id, until it has ``n_clusters`` nodes;
* slices: recursive bisection of the 6-D vectors (p / diag, 0.5 n) along the
  widest axis, at the count median (equal slices) or at the midpoint
  (uneven slices, leaf <= ``slice_max``); the batching workload instead cuts
  a Morton-ordered pixel run into slices of log-uniform sizes.
"""
from __future__ import annotations

import dataclasses
import heapq
import math

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class SceneConfig:
    name: str
    width: int
    height: int
    region_w: float
    n_spheres: int
    n_vpls: int
    n_clusters: int
    phong_prob: float
    rank: int
    slice_mode: str            # "equal", "uneven" or "batch"
    n_slices: int = 0          # equal mode: number of slices (power of two)
    slice_max: int = 1024      # uneven mode: largest leaf
    pass1_ppm: int = 50000
    pass2_ppm: int = 50000
    # batch mode only
    batch_slices: int = 0
    batch_m: tuple = (64, 4096)
    batch_n: tuple = (256, 2048)
    batch_q: tuple = (4, 8, 16, 32)
    # "spheres", or "triangles": every sphere tessellated into an icosphere of
    # 20 4^mesh_level faces on a two-triangle ground plane, and the VPLs from
    # instant radiosity (first bounces of paths from a disk light above)
    geometry: str = "spheres"
    mesh_level: int = 2

    @property
    def m(self):
        return self.width * self.height


CONFIGS = {
    # 64x64 points, 32 spheres, 1,024 VPLs as singleton clusters, 16 slices
    # of 256, rank 8, Lambertian, 5% uniform + 5% importance.
    "tiny": SceneConfig("tiny", 64, 64, 1.0, 32, 1024, 1024, 0.0, 8, "equal",
                        n_slices=16, pass1_ppm=50000, pass2_ppm=50000),
    # 512x512 points, 512 spheres, 65,536 VPLs cut to 4,096 clusters, 256
    # slices of 1,024, rank 16, half of the objects Phong; 1/5/10% rates.
    "mid": SceneConfig("mid", 512, 512, 1.0, 512, 65536, 4096, 0.5, 16, "equal",
                       n_slices=256, pass1_ppm=25000, pass2_ppm=25000),
    # 1,024 slices of log-uniform rows [64, 4096], per-slice cuts
    # log-uniform [256, 2048], ranks in {4, 8, 16, 32}; 5% sampling.
    "batch": SceneConfig("batch", 1920, 1080, 16.0 / 9.0, 2048, 300000, 2048, 1.0, 0, "batch",
                         batch_slices=1024, pass1_ppm=25000, pass2_ppm=25000),
    # 16 slices of 256 points per scene, like "tiny" but half of the objects
    # Phong; the learned-proposal training, validation and held-out scenes.
    "learned": SceneConfig("learned", 64, 64, 1.0, 32, 1024, 1024, 0.5, 8, "equal",
                           n_slices=16, pass1_ppm=50000, pass2_ppm=50000),
    # 1920x1080, 2,048 spheres, 300,000 VPLs cut to 16,384 clusters, uneven
    # slices of at most 1,024 points, all Phong, rank 32 (16 below 512 rows).
    "frame": SceneConfig("frame", 1920, 1080, 16.0 / 9.0, 2048, 300000, 16384, 1.0, 32, "uneven",
                         slice_max=1024, pass1_ppm=25000, pass2_ppm=25000),
    # triangle scenes: "tiny" and "mid" with the spheres as meshes (10,242 and
    # 163,842 triangles) and instant-radiosity VPLs
    "tri": SceneConfig("tri", 64, 64, 1.0, 32, 1024, 1024, 0.5, 8, "equal",
                       n_slices=16, pass1_ppm=50000, pass2_ppm=50000, geometry="triangles"),
    "trimid": SceneConfig("trimid", 512, 512, 1.0, 512, 65536, 4096, 0.5, 16, "equal",
                          n_slices=256, pass1_ppm=25000, pass2_ppm=25000, geometry="triangles"),
}


@dataclasses.dataclass
class Scene:
    """Structure-of-arrays scene: every float array is float32, every index int32."""
    cfg: SceneConfig
    seed: int
    points: dict          # px py pz nx ny nz kd_r kd_g kd_b ks phong_e ; object id in "obj"
    vpls: dict            # x y z nx ny nz ir ig ib
    spheres: dict         # cx cy cz r
    cut_offsets: np.ndarray
    cut_members: np.ndarray
    pt_offsets: np.ndarray
    pt_ids: np.ndarray
    cl_offsets: np.ndarray
    cl_ids: np.ndarray
    rank: np.ndarray
    # the light tree above the cut (left/right children of the n_c - 1 split
    # nodes, ids as in tree_above_cut); None where the slices have their own cuts
    tree_left: np.ndarray = None
    tree_right: np.ndarray = None

    @property
    def m(self):
        return int(self.points["px"].shape[0])

    @property
    def n(self):
        return int(self.vpls["x"].shape[0])

    @property
    def n_clusters(self):
        return int(self.cut_offsets.shape[0] - 1)

    @property
    def n_slices(self):
        return int(self.pt_offsets.shape[0] - 1)

    def slice_rows(self, s):
        return self.pt_ids[self.pt_offsets[s]:self.pt_offsets[s + 1]]

    def slice_cols(self, s):
        return self.cl_ids[self.cl_offsets[s]:self.cl_offsets[s + 1]]


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def _spheres(rng, n, region_w):
    r = rng.uniform(0.02, 0.1, n)
    cx = rng.uniform(0.0, region_w, n)
    cy = rng.uniform(0.0, 1.0, n)
    return cx, cy, r.copy(), r


def _camera_hits(width, height, region_w, cx, cy, cz, r):
    """Nearest hit of the vertical primary rays; returns positions, normals, object id."""
    xs = (np.arange(width, dtype=np.float64) + 0.5) * (region_w / width)
    ys = (np.arange(height, dtype=np.float64) + 0.5) / height
    X, Y = np.meshgrid(xs, ys)           # row-major: v (y) outer, u (x) inner
    X = X.ravel()
    Y = Y.ravel()
    Z = np.zeros_like(X)
    obj = np.zeros(X.shape, dtype=np.int32)
    dx_pix = region_w / width
    dy_pix = 1.0 / height
    for k in range(cx.shape[0]):
        u0 = max(0, int(math.floor((cx[k] - r[k]) / dx_pix - 0.5)) - 1)
        u1 = min(width - 1, int(math.ceil((cx[k] + r[k]) / dx_pix - 0.5)) + 1)
        v0 = max(0, int(math.floor((cy[k] - r[k]) / dy_pix - 0.5)) - 1)
        v1 = min(height - 1, int(math.ceil((cy[k] + r[k]) / dy_pix - 0.5)) + 1)
        if u1 < u0 or v1 < v0:
            continue
        vv, uu = np.meshgrid(np.arange(v0, v1 + 1), np.arange(u0, u1 + 1), indexing="ij")
        idx = (vv * width + uu).ravel()
        d2 = (X[idx] - cx[k]) ** 2 + (Y[idx] - cy[k]) ** 2
        inside = d2 < r[k] * r[k]
        idx = idx[inside]
        z = cz[k] + np.sqrt(r[k] * r[k] - d2[inside])
        closer = z > Z[idx]
        idx = idx[closer]
        Z[idx] = z[closer]
        obj[idx] = k + 1
    N = np.zeros((X.shape[0], 3))
    N[:, 2] = 1.0
    on_s = obj > 0
    k = obj[on_s] - 1
    N[on_s, 0] = (X[on_s] - cx[k]) / r[k]
    N[on_s, 1] = (Y[on_s] - cy[k]) / r[k]
    N[on_s, 2] = (Z[on_s] - cz[k]) / r[k]
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return X, Y, Z, N, obj


def icosphere(level):
    """Unit icosphere: vertices (V, 3) on the unit sphere and faces (F, 3),
    F = 20 4^level, every face wound counter-clockwise seen from outside."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0), (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    V = [np.asarray(v, np.float64) / math.sqrt(1.0 + g * g) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                mid[key] = len(V) - 1
            return mid[key]

        F2 = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    V = np.asarray(V)
    F = np.asarray(F, np.int64)
    # outward winding: the face normal points away from the centre
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("fk,fk->f", n, V[F].mean(axis=1)) < 0.0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def _meshes(cx, cy, cz, r, level, region_w):
    """Triangles (T, 3, 3) of the icospheres and the ground plane (two faces
    covering the image region with a margin), their object ids (0 is the
    ground) and unit face normals."""
    V, F = icosphere(level)
    tri = (np.stack([cx, cy, cz], axis=1)[:, None, None, :] + r[:, None, None, None] * V[F][None]).reshape(-1, 3, 3)
    obj = np.repeat(np.arange(1, cx.shape[0] + 1), F.shape[0])
    x0, x1, y0, y1 = -1.0, region_w + 1.0, -1.0, 2.0
    ground = np.array([[[x0, y0, 0.0], [x1, y0, 0.0], [x1, y1, 0.0]], [[x0, y0, 0.0], [x1, y1, 0.0], [x0, y1, 0.0]]])
    tri = np.concatenate([ground, tri])
    obj = np.concatenate([[0, 0], obj])
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return tri, obj, n, F.shape[0]


def _camera_hits_mesh(width, height, region_w, cx, cy, r, tri, nrm, per):
    """Nearest hit of the vertical primary rays on the meshes: for each pixel
    inside a sphere's disc, the highest point of the sphere's faces above it
    (barycentric coordinates in the image plane), else the ground."""
    xs = (np.arange(width, dtype=np.float64) + 0.5) * (region_w / width)
    ys = (np.arange(height, dtype=np.float64) + 0.5) / height
    X, Y = np.meshgrid(xs, ys)
    X = X.ravel()
    Y = Y.ravel()
    Z = np.zeros_like(X)
    N = np.zeros((X.shape[0], 3))
    N[:, 2] = 1.0
    obj = np.zeros(X.shape, dtype=np.int32)
    dx_pix = region_w / width
    dy_pix = 1.0 / height
    for k in range(cx.shape[0]):
        u0 = max(0, int(math.floor((cx[k] - r[k]) / dx_pix - 0.5)) - 1)
        u1 = min(width - 1, int(math.ceil((cx[k] + r[k]) / dx_pix - 0.5)) + 1)
        v0 = max(0, int(math.floor((cy[k] - r[k]) / dy_pix - 0.5)) - 1)
        v1 = min(height - 1, int(math.ceil((cy[k] + r[k]) / dy_pix - 0.5)) + 1)
        if u1 < u0 or v1 < v0:
            continue
        vv, uu = np.meshgrid(np.arange(v0, v1 + 1), np.arange(u0, u1 + 1), indexing="ij")
        idx = (vv * width + uu).ravel()
        T = tri[2 + k * per: 2 + (k + 1) * per]
        up = nrm[2 + k * per: 2 + (k + 1) * per, 2] > 0.0          # faces seen from above
        T = T[up]
        fn = nrm[2 + k * per: 2 + (k + 1) * per][up]
        a, b, c = T[:, 0], T[:, 1], T[:, 2]
        px = X[idx][:, None]
        py = Y[idx][:, None]
        den = (b[:, 1] - c[:, 1]) * (a[:, 0] - c[:, 0]) + (c[:, 0] - b[:, 0]) * (a[:, 1] - c[:, 1])
        l0 = ((b[:, 1] - c[:, 1]) * (px - c[:, 0]) + (c[:, 0] - b[:, 0]) * (py - c[:, 1])) / den
        l1 = ((c[:, 1] - a[:, 1]) * (px - c[:, 0]) + (a[:, 0] - c[:, 0]) * (py - c[:, 1])) / den
        l2 = 1.0 - l0 - l1
        inside = (l0 >= 0.0) & (l1 >= 0.0) & (l2 >= 0.0)
        z = np.where(inside, l0 * a[:, 2] + l1 * b[:, 2] + l2 * c[:, 2], -np.inf)
        best = np.argmax(z, axis=1)
        zb = z[np.arange(idx.shape[0]), best]
        hit = zb > Z[idx]
        idx, best, zb = idx[hit], best[hit], zb[hit]
        Z[idx] = zb
        N[idx] = fn[best]
        obj[idx] = k + 1
    return X, Y, Z, N, obj


def _first_hits(o, d, tri, nrm, cx, cy, cz, r, per):
    """Nearest hit (t > 0) of rays o + t d on the meshes; the icospheres are
    inscribed in their spheres, so only rays meeting a sphere are tested
    against its faces.  Returns t (inf for a miss) and the face index."""
    E = o.shape[0]
    best_t = np.full(E, np.inf)
    best_f = np.full(E, -1, np.int64)

    def test(rows, faces):
        if rows.size == 0 or faces.size == 0:
            return
        T = tri[faces]
        e1 = T[:, 1] - T[:, 0]
        e2 = T[:, 2] - T[:, 0]
        D = d[rows]
        p = np.cross(D[:, None, :], e2[None])
        det = np.einsum("etk,tk->et", p, e1)
        sv = o[rows][:, None, :] - T[None, :, 0]
        q = np.cross(sv, e1[None])
        with np.errstate(divide="ignore", invalid="ignore"):
            u = np.einsum("etk,etk->et", sv, p) / det
            v = np.einsum("ek,etk->et", D, q) / det
            t = np.einsum("tk,etk->et", e2, q) / det
        ok = (det != 0.0) & (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t > 1e-9)
        t = np.where(ok, t, np.inf)
        k = np.argmin(t, axis=1)
        tk = t[np.arange(rows.shape[0]), k]
        better = tk < best_t[rows]
        best_t[rows[better]] = tk[better]
        best_f[rows[better]] = faces[k[better]]

    test(np.arange(E), np.array([0, 1]))
    c = np.stack([cx, cy, cz], axis=1)
    for s0 in range(0, c.shape[0], 256):
        cs = c[s0:s0 + 256]
        oc = cs[None, :, :] - o[:, None, :]
        tc = np.einsum("esk,ek->es", oc, d)
        dist2 = np.einsum("esk,esk->es", oc, oc) - tc * tc
        near = (dist2 <= (r[s0:s0 + 256] ** 2)[None, :]) & (tc > -r[s0:s0 + 256][None, :])
        for j in np.unique(np.nonzero(near)[1]):
            k = s0 + j
            rows = np.nonzero(near[:, j])[0]
            test(rows, np.arange(2 + k * per, 2 + (k + 1) * per))
    return best_t, best_f


def _ir_vpls(rng, n, region_w, tri, nrm, obj, kd, cx, cy, cz, r, per):
    """Instant radiosity: n paths from a downward-facing disk light (radius
    0.3, height 2, unit white power, cosine emission); the first hit of each
    path on a face becomes a VPL with that face's normal, lifted 2e-3 off it,
    carrying power 1/n times the face's diffuse albedo.  Paths that leave
    the scene are drawn again."""
    X = np.zeros((0, 3))
    Nn = np.zeros((0, 3))
    C = np.zeros((0, 3))
    while X.shape[0] < n:
        k = 2 * (n - X.shape[0]) + 64
        a = rng.uniform(0.0, 1.0, k)
        ph = rng.uniform(0.0, 2.0 * math.pi, k)
        rad = 0.3 * np.sqrt(a)
        o = np.stack([0.5 * region_w + rad * np.cos(ph), 0.5 + rad * np.sin(ph), np.full(k, 2.0)], axis=1)
        u1 = rng.uniform(0.0, 1.0, k)
        u2 = rng.uniform(0.0, 2.0 * math.pi, k)
        sr = np.sqrt(u1)
        d = np.stack([sr * np.cos(u2), sr * np.sin(u2), -np.sqrt(np.maximum(0.0, 1.0 - u1))], axis=1)
        t, f = _first_hits(o, d, tri, nrm, cx, cy, cz, r, per)
        p = o + np.where(np.isfinite(t), t, 0.0)[:, None] * d
        inside = np.isfinite(t) & (p[:, 0] >= 0.0) & (p[:, 0] <= region_w) & (p[:, 1] >= 0.0) & (p[:, 1] <= 1.0)
        f = f[inside]
        X = np.concatenate([X, p[inside] + 2e-3 * nrm[f]])
        Nn = np.concatenate([Nn, nrm[f]])
        C = np.concatenate([C, kd[obj[f]]])
    X, Nn, C = X[:n], Nn[:n], C[:n]
    return X[:, 0], X[:, 1], X[:, 2], Nn, C / n * 1000.0


def _materials(rng, n_obj, phong_prob):
    albedo = rng.uniform(0.2, 0.9, (n_obj, 3))
    is_phong = rng.uniform(0.0, 1.0, n_obj) < phong_prob
    expo = rng.uniform(10.0, 100.0, n_obj)
    kd = np.where(is_phong[:, None], 0.75 * albedo, albedo)
    ks = np.where(is_phong, 0.2, 0.0)
    e = np.where(is_phong, expo, 1.0)
    return kd, ks, e


def _vpls(rng, n, region_w):
    x = rng.uniform(0.0, region_w, n)
    y = rng.uniform(0.0, 1.0, n)
    z = rng.uniform(0.25, 1.0, n)
    u1 = rng.uniform(0.0, 1.0, n)
    u2 = rng.uniform(0.0, 1.0, n)
    rr = np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    d = np.stack([rr * np.cos(phi), rr * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    nrm = -d
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    return x, y, z, nrm, rgb


# ----------------------------------------------------------------------------
# light tree cut
# ----------------------------------------------------------------------------

def light_tree_cut_sequence(pos, rgb, max_clusters):
    """Grow a light-tree cut greedily; returns the list of nodes (member arrays,
    ascending VPL ids) in creation order plus the sequence of cuts as sets of
    node ids: ``cuts[k]`` is the cut with k+1 nodes."""
    n = pos.shape[0]
    nodes = [np.arange(n, dtype=np.int64)]
    weight = []

    def w_of(members):
        if members.shape[0] < 2:
            return 0.0
        p = pos[members]
        diag = float(np.linalg.norm(p.max(axis=0) - p.min(axis=0)))
        return float(rgb[members].sum()) * diag

    heap = [(-w_of(nodes[0]), 0)]
    cut = {0}
    history = []
    children = {}
    while len(cut) < max_clusters and heap:
        negw, nid = heapq.heappop(heap)
        members = nodes[nid]
        if members.shape[0] < 2:
            break
        p = pos[members]
        axis = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
        order = np.argsort(p[:, axis], kind="stable")
        half = members.shape[0] // 2
        left = np.sort(members[order[:half]])
        right = np.sort(members[order[half:]])
        cut.discard(nid)
        kids = []
        for ch in (left, right):
            nodes.append(ch)
            cid = len(nodes) - 1
            cut.add(cid)
            kids.append(cid)
            heapq.heappush(heap, (-w_of(ch), cid))
        children[nid] = tuple(kids)
        history.append(sorted(cut))
    del weight
    light_tree_cut_sequence.children = children
    return nodes, history, sorted(cut)


def tree_above_cut(children, cut_node_order):
    """The light tree's nodes above a cut as a binary tree over the cut's
    clusters: cluster k (cut-table order) is node k; the n_c - 1 split nodes
    are nodes n_c .. 2 n_c - 2, children before parents (the root last).
    Returns (left, right) int32 arrays of the split nodes' children."""
    nc = len(cut_node_order)
    ids = {nid: k for k, nid in enumerate(cut_node_order)}
    split = sorted(children, reverse=True)        # created later -> deeper -> first
    for k, nid in enumerate(split):
        ids[nid] = nc + k
    left = np.array([ids[children[nid][0]] for nid in split], dtype=np.int32)
    right = np.array([ids[children[nid][1]] for nid in split], dtype=np.int32)
    return left, right


def full_light_tree(pos):
    """The light tree over every VPL, grown to single lights by the same split
    as light_tree_cut_sequence (median along the longest axis of the members'
    box, members taken by ascending id before a stable sort), so any cut that
    sequence makes is a cut of this tree.

    Layout: leaves 0 .. n-1 are the VPLs perm[0 .. n) in an order where every
    node's leaves are contiguous (left child's before right child's); split
    node n + k has children left[k], right[k], children before parents, the
    root 2 n - 2.  Returns (perm, left, right) as int32 arrays."""
    pos = np.asarray(pos, np.float64)
    n = pos.shape[0]
    perm = np.arange(n, dtype=np.int64)
    if n < 2:
        return perm.astype(np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32)
    # internal nodes are numbered breadth-first (root 0) while growing; BFS id
    # b is node n + (n - 2 - b), so children precede parents and the root is last
    L = np.zeros(n - 1, np.int64)
    R = np.zeros(n - 1, np.int64)
    starts = np.array([0], np.int64)
    sizes = np.array([n], np.int64)
    ids = np.array([0], np.int64)     # BFS id of each segment of this level
    next_id = 1
    while starts.size:
        first = np.cumsum(sizes) - sizes
        seg = np.repeat(np.arange(starts.size), sizes)
        idx = np.arange(int(sizes.sum())) + np.repeat(starts - first, sizes)
        p = pos[perm[idx]]
        lo = np.minimum.reduceat(p, first, axis=0)
        hi = np.maximum.reduceat(p, first, axis=0)
        axis = np.argmax(hi - lo, axis=1)
        coord = p[np.arange(idx.size), axis[seg]]
        order = np.lexsort((perm[idx], coord, seg))
        perm[idx] = perm[idx][order]
        half = sizes // 2
        c_st = np.stack([starts, starts + half], axis=1).ravel()
        c_sz = np.stack([half, sizes - half], axis=1).ravel()
        inner = c_sz > 1
        c_bfs = next_id + np.cumsum(inner) - 1
        next_id += int(inner.sum())
        c_node = np.where(inner, n + (n - 2 - c_bfs), c_st)
        k = (n - 2) - ids
        L[k] = c_node[0::2]
        R[k] = c_node[1::2]
        starts, sizes, ids = c_st[inner], c_sz[inner], c_bfs[inner]
    assert next_id == n - 1
    return perm.astype(np.int32), L.astype(np.int32), R.astype(np.int32)


def _cut_table(nodes, node_ids):
    """Cut as CSR: clusters ordered by their smallest member id."""
    node_ids = sorted(node_ids, key=lambda i: int(nodes[i][0]))
    offsets = np.zeros(len(node_ids) + 1, dtype=np.int64)
    for k, i in enumerate(node_ids):
        offsets[k + 1] = offsets[k] + nodes[i].shape[0]
    members = np.concatenate([nodes[i] for i in node_ids]) if node_ids else np.zeros(0, np.int64)
    return offsets.astype(np.int32), members.astype(np.int32), node_ids


# ----------------------------------------------------------------------------
# slices
# ----------------------------------------------------------------------------

def _bisect_slices(feat, ids, mode, n_leaves=None, leaf_max=None):
    out = []

    def rec(sub, depth_left):
        if mode == "equal":
            if depth_left == 0:
                out.append(np.sort(sub))
                return
        else:
            if sub.shape[0] <= leaf_max:
                out.append(np.sort(sub))
                return
        f = feat[sub]
        ext = f.max(axis=0) - f.min(axis=0)
        axis = int(np.argmax(ext))
        if mode == "equal":
            order = np.argsort(f[:, axis], kind="stable")
            half = sub.shape[0] // 2
            a, b = sub[order[:half]], sub[order[half:]]
        else:
            mid = 0.5 * (f[:, axis].max() + f[:, axis].min())
            left = f[:, axis] < mid
            if left.all() or (~left).all():
                order = np.argsort(f[:, axis], kind="stable")
                half = sub.shape[0] // 2
                a, b = sub[order[:half]], sub[order[half:]]
            else:
                a, b = sub[left], sub[~left]
        rec(a, None if depth_left is None else depth_left - 1)
        rec(b, None if depth_left is None else depth_left - 1)

    if mode == "equal":
        depth = int(round(math.log2(n_leaves)))
        assert 1 << depth == n_leaves
        rec(ids, depth)
    else:
        rec(ids, None)
    return out


def _morton(width, height):
    u = np.tile(np.arange(width), height)
    v = np.repeat(np.arange(height), width)

    def spread(x):
        x = x.astype(np.uint64)
        r = np.zeros_like(x)
        for b in range(16):
            r |= ((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        return r
    return spread(u) | (spread(v) << np.uint64(1))


# ----------------------------------------------------------------------------
# entry point
# ----------------------------------------------------------------------------

def supported_rank(q, limit):
    """The largest completion rank in {4, 8, 16, 32} that is at most both q and
    limit (a slice's rows or columns), elementwise; limit below 4 keeps limit."""
    q = np.minimum(np.asarray(q, np.int64), np.asarray(limit, np.int64))
    out = np.where(q >= 32, 32, np.where(q >= 16, 16, np.where(q >= 8, 8, np.where(q >= 4, 4, q))))
    return out.astype(np.int32)


def make_scene(cfg, seed, n_vpls=None, n_clusters=None):
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    rng = np.random.default_rng(seed)
    n_vpls = cfg.n_vpls if n_vpls is None else n_vpls
    n_clusters = cfg.n_clusters if n_clusters is None else n_clusters

    cx, cy, cz, r = _spheres(rng, cfg.n_spheres, cfg.region_w)
    if cfg.geometry == "triangles":
        tri, tri_obj, tri_n, per = _meshes(cx, cy, cz, r, cfg.mesh_level, cfg.region_w)
        X, Y, Z, N, obj = _camera_hits_mesh(cfg.width, cfg.height, cfg.region_w, cx, cy, r, tri, tri_n, per)
    else:
        X, Y, Z, N, obj = _camera_hits(cfg.width, cfg.height, cfg.region_w, cx, cy, cz, r)
    kd, ks, e = _materials(rng, cfg.n_spheres + 1, cfg.phong_prob)
    points = dict(px=X, py=Y, pz=Z, nx=N[:, 0], ny=N[:, 1], nz=N[:, 2],
                  kd_r=kd[obj, 0], kd_g=kd[obj, 1], kd_b=kd[obj, 2], ks=ks[obj], phong_e=e[obj])
    points = {k: v.astype(F32) for k, v in points.items()}
    points["obj"] = obj.astype(np.int32)

    if cfg.geometry == "triangles":
        vx, vy, vz, vn, vrgb = _ir_vpls(rng, n_vpls, cfg.region_w, tri, tri_n, tri_obj, kd, cx, cy, cz, r, per)
    else:
        vx, vy, vz, vn, vrgb = _vpls(rng, n_vpls, cfg.region_w)
    vpls = dict(x=vx, y=vy, z=vz, nx=vn[:, 0], ny=vn[:, 1], nz=vn[:, 2],
                ir=vrgb[:, 0], ig=vrgb[:, 1], ib=vrgb[:, 2])
    vpls = {k: v.astype(F32) for k, v in vpls.items()}
    if cfg.geometry == "triangles":
        # the occluders: (T, 9) FP32 vertices (v0, v1, v2) under the key "tri"
        spheres = {"tri": tri.reshape(-1, 9).astype(F32)}
    else:
        spheres = {k: v.astype(F32) for k, v in dict(cx=cx, cy=cy, cz=cz, r=r).items()}

    vpos = np.stack([vpls["x"], vpls["y"], vpls["z"]], axis=1).astype(np.float64)
    vrgb64 = np.stack([vpls["ir"], vpls["ig"], vpls["ib"]], axis=1).astype(np.float64)
    m = cfg.m
    pts_pos = np.stack([points["px"], points["py"], points["pz"]], axis=1).astype(np.float64)
    pts_nrm = np.stack([points["nx"], points["ny"], points["nz"]], axis=1).astype(np.float64)
    diag = float(np.linalg.norm(pts_pos.max(axis=0) - pts_pos.min(axis=0)))
    feat = np.concatenate([pts_pos / diag, 0.5 * pts_nrm], axis=1)

    tree_left = tree_right = None
    if cfg.slice_mode in ("equal", "uneven"):
        # a cut of every VPL is the tree grown down to single lights
        nodes, _, final = light_tree_cut_sequence(vpos, vrgb64, min(n_clusters, n_vpls))
        children = light_tree_cut_sequence.children
        cut_offsets, cut_members, order = _cut_table(nodes, final)
        tree_left, tree_right = tree_above_cut(children, order)
        ids = np.arange(m, dtype=np.int64)
        if cfg.slice_mode == "equal":
            leaves = _bisect_slices(feat, ids, "equal", n_leaves=cfg.n_slices)
        else:
            leaves = _bisect_slices(feat, ids, "uneven", leaf_max=cfg.slice_max)
        S = len(leaves)
        nc = cut_offsets.shape[0] - 1
        pt_offsets = np.zeros(S + 1, dtype=np.int64)
        for s, lf in enumerate(leaves):
            pt_offsets[s + 1] = pt_offsets[s] + lf.shape[0]
        pt_ids = np.concatenate(leaves)
        cl_offsets = np.arange(S + 1, dtype=np.int64) * nc
        cl_ids = np.tile(np.arange(nc, dtype=np.int64), S)
        if cfg.slice_mode == "equal":
            rank = np.full(S, cfg.rank, dtype=np.int32)
        else:
            sizes = np.diff(pt_offsets)
            rank = np.where(sizes >= 512, cfg.rank, min(cfg.rank, 16)).astype(np.int32)
            rank = supported_rank(rank, np.minimum(sizes, nc))
    else:  # batch: per-slice cuts from one greedy growth sequence
        S = cfg.batch_slices
        lo_m, hi_m = cfg.batch_m
        lo_n, hi_n = cfg.batch_n
        ms = np.exp(rng.uniform(math.log(lo_m), math.log(hi_m), S)).astype(np.int64)
        ns = np.exp(rng.uniform(math.log(lo_n), math.log(hi_n), S)).astype(np.int64)
        qs = rng.choice(np.asarray(cfg.batch_q), S).astype(np.int32)
        ms = np.clip(ms, lo_m, hi_m)
        ns = np.clip(ns, lo_n, hi_n)
        total = int(ms.sum())
        if total > m:
            raise ValueError("batch slices exceed the image")
        order = np.argsort(_morton(cfg.width, cfg.height), kind="stable")
        nodes, history, _ = light_tree_cut_sequence(vpos, vrgb64, int(ns.max()))
        # cluster table = every node that appears in some slice's cut
        used = sorted({nid for s in range(S) for nid in history[int(ns[s]) - 2]})
        cut_offsets, cut_members, node_order = _cut_table(nodes, used)
        pos_of = {nid: k for k, nid in enumerate(node_order)}
        pt_offsets = np.zeros(S + 1, dtype=np.int64)
        cl_offsets = np.zeros(S + 1, dtype=np.int64)
        pt_list, cl_list = [], []
        start = 0
        for s in range(S):
            pt_list.append(np.sort(order[start:start + ms[s]]))
            start += int(ms[s])
            cut_s = sorted((pos_of[nid] for nid in history[int(ns[s]) - 2]))
            cl_list.append(np.asarray(cut_s, dtype=np.int64))
            pt_offsets[s + 1] = pt_offsets[s] + ms[s]
            cl_offsets[s + 1] = cl_offsets[s] + len(cut_s)
        pt_ids = np.concatenate(pt_list)
        cl_ids = np.concatenate(cl_list)
        rank = np.minimum(qs, np.minimum(ms, ns)).astype(np.int32)

    return Scene(cfg=cfg, seed=seed, points=points, vpls=vpls, spheres=spheres,
                 cut_offsets=np.asarray(cut_offsets, dtype=np.int32),
                 cut_members=np.asarray(cut_members, dtype=np.int32),
                 pt_offsets=pt_offsets.astype(np.int32), pt_ids=pt_ids.astype(np.int32),
                 cl_offsets=cl_offsets.astype(np.int32), cl_ids=cl_ids.astype(np.int32),
                 rank=np.asarray(rank, dtype=np.int32), tree_left=tree_left, tree_right=tree_right)


def scene_sample(scene: Scene, slices):
    """A scene restricted to a subset of its slices (same points, VPLs, cut):
    used to time the oracle on a bounded sample of a large workload."""
    slices = list(slices)
    pt = [scene.slice_rows(s) for s in slices]
    cl = [scene.slice_cols(s) for s in slices]
    pt_offsets = np.concatenate([[0], np.cumsum([a.shape[0] for a in pt])]).astype(np.int32)
    cl_offsets = np.concatenate([[0], np.cumsum([a.shape[0] for a in cl])]).astype(np.int32)
    return dataclasses.replace(scene, pt_offsets=pt_offsets, pt_ids=np.concatenate(pt).astype(np.int32),
                               cl_offsets=cl_offsets, cl_ids=np.concatenate(cl).astype(np.int32),
                               rank=scene.rank[slices].copy())
