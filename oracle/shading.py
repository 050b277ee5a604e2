"""Lighting-matrix entries A(i, j): contribution of light j to surface point i
(Sec. 3, matrix formulation), with shadow-ray visibility, which the paper
names the most expensive part of an entry (Sec. 2, many-light methods;
Sec. 6 ray casting).  The paper does not print the shading model; this is
the standard VPL contribution, our reading:

    d = y - x,  r^2 = d.d,  w = d / r
    c_x = n_x . w,  c_y = -n_y . w          (0 if either is <= 0: no ray)
    G = c_x c_y / max(r^2, r_min^2)          (clamped geometry term)
    f = rho_d / pi + rho_s (e + 2) / (2 pi) max(0, w_r . w_o)^e,
        w_r = 2 (n_x . w) n_x - w            (normalised Phong; rho_s = 0: Lambertian)
    A = f * I * G * V

V = 1 iff the segment from o = x + eps n_x to y meets no sphere, i.e. for
every sphere (c, r) the distance from c to the segment is >= r.  Both
endpoints lie outside every sphere by construction of the scenes, so this
is the same as "no hit at t in (0, 1)".

Visibility is decided here in FP64 by brute force over every sphere (no
acceleration structure).  An entry is flagged *ambiguous* when a
perturbation of AMBIG in some sphere distance could flip V; parity tests
compare only unflagged entries and count the flagged ones.

Triangle occluders (the paper's scenes are triangle meshes traced through an
SBVH, Sec. 6): V = 0 iff the open segment meets a triangle, decided by the
barycentric coordinates (u, v) and the segment parameter t of the crossing
with the triangle's plane, again by brute force; the ambiguity flag uses a
margin AMBIG_TRI on those parameters.

Pinned by: closed forms for unoccluded point-to-point configurations and
analytic occluded/unoccluded segment-sphere cases
(tests/test_oracle_shading.py).
"""
import numpy as np

AMBIG = 1e-5
AMBIG_TRI = 1e-4
INV_PI = 1.0 / np.pi


def segment_sphere_dist(o, D, c):
    """Distance from sphere centres c (S, 3) to segments o + t D, t in [0, 1];
    o, D are (E, 3).  Returns (E, S)."""
    oc = c[None, :, :] - o[:, None, :]                      # (E, S, 3)
    dd = np.einsum("ek,ek->e", D, D)[:, None]
    t = np.clip(np.einsum("esk,ek->es", oc, D) / dd, 0.0, 1.0)
    p = o[:, None, :] + t[:, :, None] * D[:, None, :] - c[None, :, :]
    return np.sqrt(np.einsum("esk,esk->es", p, p))


def segment_triangle(o, D, v0, v1, v2):
    """Segments o + t D (E, 3) against triangles (T, 3) by the barycentric
    form of the intersection (Moller-Trumbore): returns the margins (E, T) of
    the four conditions u >= 0, v >= 0, u + v <= 1 and 0 < t < 1 (their
    minimum: positive inside, negative outside; -inf where the segment is
    parallel to the triangle's plane) and the plane-angle term |det| /
    (|D| |e1| |e2|) (E, T)."""
    e1 = v1 - v0
    e2 = v2 - v0
    p = np.cross(D[:, None, :], e2[None, :, :])                 # (E, T, 3)
    det = np.einsum("etk,tk->et", p, e1)
    s = o[:, None, :] - v0[None, :, :]
    q = np.cross(s, e1[None, :, :])
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        u = np.einsum("etk,etk->et", s, p) * inv
        v = np.einsum("ek,etk->et", D, q) * inv
        t = np.einsum("tk,etk->et", e2, q) * inv
        margin = np.minimum(np.minimum(u, v), np.minimum(1.0 - u - v, np.minimum(t, 1.0 - t)))
    scale = (np.linalg.norm(D, axis=1)[:, None] * np.linalg.norm(e1, axis=1)[None, :]
             * np.linalg.norm(e2, axis=1)[None, :])
    angle = np.abs(det) / scale
    margin = np.where(det != 0.0, margin, -np.inf)
    return margin, angle


def triangle_visibility(o, y, tri, chunk=1 << 22):
    """V (E,) and an ambiguity flag (E,) for segments o -> y against
    triangles tri (T, 9) = (v0, v1, v2): V = 0 iff some triangle is met at a
    parameter t in (0, 1), brute force over every triangle.  A pair is
    ambiguous when no triangle blocks it by more than AMBIG_TRI (in the
    barycentric and segment parameters) but one comes within AMBIG_TRI of
    blocking it, or when a triangle within reach is nearly parallel to the
    segment (angle term below AMBIG_TRI)."""
    tri = np.asarray(tri, np.float64).reshape(-1, 9)
    v0, v1, v2 = tri[:, 0:3], tri[:, 3:6], tri[:, 6:9]
    E = o.shape[0]
    V = np.ones(E)
    amb = np.zeros(E, dtype=bool)
    if tri.shape[0] == 0:
        return V, amb
    step = max(1, chunk // max(1, tri.shape[0]))
    for a in range(0, E, step):
        b = min(E, a + step)
        margin, angle = segment_triangle(o[a:b], y[a:b] - o[a:b], v0, v1, v2)
        blocked = (margin > 0.0).any(axis=1)
        sure = (margin > AMBIG_TRI).any(axis=1)
        near = ((np.abs(margin) < AMBIG_TRI) | ((angle < AMBIG_TRI) & (margin > -AMBIG_TRI))).any(axis=1)
        V[a:b] = np.where(blocked, 0.0, 1.0)
        amb[a:b] = near & ~sure
    return V, amb


def visibility(o, y, spheres, chunk=4096):
    """V (E,) in {0, 1} and an ambiguity flag (E,) for segments o -> y; the
    occluders are spheres (cx, cy, cz, r) or, with key "tri", triangles."""
    if "tri" in spheres:
        return triangle_visibility(o, y, spheres["tri"])
    c = np.stack([spheres["cx"], spheres["cy"], spheres["cz"]], axis=1).astype(np.float64)
    r = np.asarray(spheres["r"], dtype=np.float64)
    E = o.shape[0]
    V = np.ones(E)
    amb = np.zeros(E, dtype=bool)
    if c.shape[0] == 0:
        return V, amb
    step = max(1, chunk * 64 // max(1, c.shape[0]))
    for a in range(0, E, step):
        b = min(E, a + step)
        dist = segment_sphere_dist(o[a:b], y[a:b] - o[a:b], c)
        margin = dist - r[None, :]
        blocked = (margin < 0.0).any(axis=1)
        sure_blocked = (margin < -AMBIG).any(axis=1)
        near = (np.abs(margin) < AMBIG).any(axis=1)
        V[a:b] = np.where(blocked, 0.0, 1.0)
        amb[a:b] = near & ~sure_blocked
    return V, amb


def entries(x, nx, kd, ks, pe, wo, y, ny, I, spheres, r_min=0.05, eps=1e-4, with_visibility=True):
    """Entry values for E (point, light) pairs, all (E, 3) / (E,) arrays.

    x, nx: point position / normal; kd: diffuse RGB; ks, pe: Phong specular
    albedo and exponent; wo: direction to the viewer; y, ny: light position /
    normal; I: light RGB intensity.  Returns (A (E, 3), ambiguous (E,),
    traced (E,)) where traced marks entries whose shadow ray was needed.
    """
    x = np.asarray(x, np.float64)
    nx = np.asarray(nx, np.float64)
    y = np.asarray(y, np.float64)
    ny = np.asarray(ny, np.float64)
    d = y - x
    r2 = np.einsum("ek,ek->e", d, d)
    r = np.sqrt(r2)
    w = d / r[:, None]
    cx = np.einsum("ek,ek->e", nx, w)
    cy = -np.einsum("ek,ek->e", ny, w)
    lit = (cx > 0.0) & (cy > 0.0)
    G = np.where(lit, cx * cy / np.maximum(r2, r_min * r_min), 0.0)
    wr = 2.0 * cx[:, None] * nx - w
    cosr = np.maximum(0.0, np.einsum("ek,ek->e", wr, np.asarray(wo, np.float64)))
    ks = np.asarray(ks, np.float64)
    pe = np.asarray(pe, np.float64)
    spec = np.where(ks > 0.0, ks * (pe + 2.0) * (0.5 * INV_PI) * cosr ** pe, 0.0)
    f = np.asarray(kd, np.float64) * INV_PI + spec[:, None]
    A = f * np.asarray(I, np.float64) * G[:, None]
    amb = np.zeros(x.shape[0], dtype=bool)
    if with_visibility and lit.any():
        idx = np.nonzero(lit)[0]
        o = x[idx] + eps * nx[idx]
        V, a = visibility(o, y[idx], spheres)
        A[idx] *= V[:, None]
        amb[idx] = a
    return A, amb, lit


def point_arrays(points, ids):
    """Gather FP64 point attributes for point ids."""
    P = points
    x = np.stack([P["px"][ids], P["py"][ids], P["pz"][ids]], axis=1).astype(np.float64)
    n = np.stack([P["nx"][ids], P["ny"][ids], P["nz"][ids]], axis=1).astype(np.float64)
    kd = np.stack([P["kd_r"][ids], P["kd_g"][ids], P["kd_b"][ids]], axis=1).astype(np.float64)
    ks = np.asarray(P["ks"][ids], np.float64)
    pe = np.asarray(P["phong_e"][ids], np.float64)
    if "vx" in P:
        wo = np.stack([P["vx"][ids], P["vy"][ids], P["vz"][ids]], axis=1).astype(np.float64)
    else:
        wo = np.zeros_like(x)
        wo[:, 2] = 1.0
    return x, n, kd, ks, pe, wo
