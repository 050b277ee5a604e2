"""Pins the oracle's entry values and visibility with closed forms.

Every expected value below is derived by hand from the geometry (comments
give the derivation), not by calling the oracle's formula again.  The
closed-form cases are also stored under tests/golden/shading_closed_form.txt.
"""
import math
import os

import numpy as np

from oracle.shading import entries, segment_sphere_dist, visibility

NO_SPHERES = dict(cx=np.zeros(0), cy=np.zeros(0), cz=np.zeros(0), r=np.zeros(0))
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "shading_closed_form.txt")


def one(x, n, kd, ks, e, wo, y, ny, I, spheres=NO_SPHERES, r_min=0.05):
    A, amb, lit = entries(np.array([x], float), np.array([n], float), np.array([kd], float),
                          np.array([ks], float), np.array([e], float), np.array([wo], float),
                          np.array([y], float), np.array([ny], float), np.array([I], float),
                          spheres, r_min=r_min)
    return A[0], bool(amb[0]), bool(lit[0])


def test_golden_closed_forms():
    with open(GOLDEN) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 6
    for r in rows:
        vals = [float(v) for v in r[1:]]
        x, n, kd, ks, e, wo, y, ny, I = (vals[0:3], vals[3:6], vals[6:9], vals[9], vals[10],
                                         vals[11:14], vals[14:17], vals[17:20], vals[20:23])
        expect = vals[23:26]
        A, _, _ = one(x, n, kd, ks, e, wo, y, ny, I)
        np.testing.assert_allclose(A, expect, rtol=1e-12, atol=1e-15, err_msg=r[0])


def test_facing_point_light_lambertian():
    # light straight above at height h, facing down: G = 1 / h^2, f = kd / pi
    for h in (0.3, 1.0, 2.5):
        A, _, lit = one([0, 0, 0], [0, 0, 1], [0.5, 0.25, 0.125], 0, 1, [0, 0, 1],
                        [0, 0, h], [0, 0, -1], [1.0, 2.0, 4.0])
        assert lit
        np.testing.assert_allclose(A, np.array([0.5, 0.5, 0.5]) / math.pi / h ** 2, rtol=1e-14)


def test_tilted_light_cosines():
    # y = (a, 0, h), both normals vertical: cos_x = cos_y = h / r, G = h^2 / r^4
    a, h = 0.6, 0.8
    r2 = a * a + h * h
    A, _, _ = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [a, 0, h], [0, 0, -1], [1, 1, 1])
    np.testing.assert_allclose(A, np.full(3, (h * h / r2 ** 2) / math.pi), rtol=1e-14)


def test_phong_peak_and_off_peak():
    # viewer along n, light along n: mirror direction = n, cos = 1
    kd, ks, e, h = 0.4, 0.2, 37.0, 0.9
    A, _, _ = one([0, 0, 0], [0, 0, 1], [kd] * 3, ks, e, [0, 0, 1], [0, 0, h], [0, 0, -1], [1, 1, 1])
    np.testing.assert_allclose(A, np.full(3, (kd / math.pi + ks * (e + 2) / (2 * math.pi)) / h ** 2), rtol=1e-14)
    # light at 45 degrees in x-z, light facing the point: mirror dir = (-s, 0, s)
    # (s = 1/sqrt2), viewer +z: cos_r = s; cos_x = cos_y = s; r = 1
    s = 1 / math.sqrt(2)
    A, _, _ = one([0, 0, 0], [0, 0, 1], [kd] * 3, ks, e, [0, 0, 1], [s, 0, s], [-s, 0, -s], [1, 1, 1])
    f = kd / math.pi + ks * (e + 2) / (2 * math.pi) * s ** e
    np.testing.assert_allclose(A, np.full(3, f * s * 1.0), rtol=1e-12)


def test_back_facing_is_zero_and_untraced():
    A, _, lit = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, -1], [0, 0, 1], [1, 1, 1])
    assert not lit and np.all(A == 0)
    A, _, lit = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, 1], [0, 0, 1], [1, 1, 1])
    assert not lit and np.all(A == 0)       # light faces away from the point


def test_clamp_binds_below_r_min():
    # r = 0.02 < r_min = 0.05: G = 1 / r_min^2 = 400
    A, _, _ = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, 0.02], [0, 0, -1], [1, 1, 1])
    np.testing.assert_allclose(A, np.full(3, 400.0 / math.pi), rtol=1e-13)


def test_occluded_and_unoccluded_segments():
    sph = dict(cx=np.array([0.0]), cy=np.array([0.0]), cz=np.array([0.5]), r=np.array([0.1]))
    A, amb, _ = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, 1], [0, 0, -1], [1, 1, 1], sph)
    assert np.all(A == 0) and not amb
    # sphere offset sideways by 0.1 + 1e-3: the vertical segment misses it
    sph2 = dict(cx=np.array([0.101]), cy=np.array([0.0]), cz=np.array([0.5]), r=np.array([0.1]))
    A, amb, _ = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, 1], [0, 0, -1], [1, 1, 1], sph2)
    assert np.all(A > 0) and not amb
    # sphere tangent within 1e-6: flagged ambiguous
    sph3 = dict(cx=np.array([0.1 + 1e-6]), cy=np.array([0.0]), cz=np.array([0.5]), r=np.array([0.1]))
    _, amb, _ = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, 1], [0, 0, -1], [1, 1, 1], sph3)
    assert amb
    # sphere beyond the light (t > 1) does not occlude
    sph4 = dict(cx=np.array([0.0]), cy=np.array([0.0]), cz=np.array([1.5]), r=np.array([0.2]))
    A, _, _ = one([0, 0, 0], [0, 0, 1], [1, 1, 1], 0, 1, [0, 0, 1], [0, 0, 1], [0, 0, -1], [1, 1, 1], sph4)
    assert np.all(A > 0)


def test_visibility_matches_quadratic_roots():
    """Textbook ray-sphere intersection (roots of |o + tD - c|^2 = r^2, hit if an
    interval root lies in (0, 1)) agrees with the oracle's distance test."""
    rng = np.random.default_rng(3)
    E, S = 2000, 24
    o = rng.uniform(0, 1, (E, 3)) * [1, 1, 0.05]
    y = rng.uniform(0, 1, (E, 3)) * [1, 1, 0.75] + [0, 0, 0.25]
    c = np.column_stack([rng.uniform(0, 1, S), rng.uniform(0, 1, S), rng.uniform(0.1, 0.2, S)])
    r = rng.uniform(0.02, 0.1, S)
    # keep endpoints outside every sphere, as the scenes guarantee
    keep = np.ones(E, bool)
    for k in range(S):
        keep &= np.linalg.norm(o - c[k], axis=1) > r[k] + 1e-3
    o, y = o[keep], y[keep]
    sph = dict(cx=c[:, 0], cy=c[:, 1], cz=c[:, 2], r=r)
    V, amb = visibility(o, y, sph)
    D = y - o
    hit = np.zeros(o.shape[0], bool)
    for k in range(S):
        oc = o - c[k]
        a = np.sum(D * D, axis=1)
        b = 2 * np.sum(oc * D, axis=1)
        cc = np.sum(oc * oc, axis=1) - r[k] ** 2
        disc = b * b - 4 * a * cc
        ok = disc > 0
        sq = np.sqrt(np.where(ok, disc, 0))
        t0 = (-b - sq) / (2 * a)
        t1 = (-b + sq) / (2 * a)
        hit |= ok & (t1 > 0) & (t0 < 1)
    sure = ~amb
    assert np.array_equal(V[sure] == 0, hit[sure])
    assert (hit.sum() > 50) and ((~hit).sum() > 50)


def test_segment_distance_closed_form():
    # centre (0.3, 0.4, 0.5) to the segment (0,0,0)-(0,0,1): distance 0.5
    d = segment_sphere_dist(np.zeros((1, 3)), np.array([[0, 0, 1.0]]), np.array([[0.3, 0.4, 0.5]]))
    np.testing.assert_allclose(d, [[0.5]], rtol=1e-15)
    # beyond the end: distance to the endpoint
    d = segment_sphere_dist(np.zeros((1, 3)), np.array([[0, 0, 1.0]]), np.array([[0.0, 0.3, 1.4]]))
    np.testing.assert_allclose(d, [[0.5]], rtol=1e-15)


# ---------------------------------------------------------------------------
# triangle occluders
# ---------------------------------------------------------------------------

from oracle.shading import AMBIG_TRI, segment_triangle, triangle_visibility  # noqa: E402

UNIT = np.array([[0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0]])


def _seg(o, y):
    return np.asarray([o], np.float64), np.asarray([y], np.float64)


def test_triangle_closed_forms():
    v0, v1, v2 = UNIT[:, 0:3], UNIT[:, 3:6], UNIT[:, 6:9]
    cases = [  # (o, y, margin): margin = min(u, v, 1 - u - v, t, 1 - t) by hand
        ((0.2, 0.2, 1.0), (0.2, 0.2, -1.0), 0.2),      # through: u = v = 0.2, t = 0.5
        ((0.1, 0.3, 2.0), (0.1, 0.3, -2.0), 0.1),      # u = 0.1 is the tightest
        ((0.6, 0.6, 1.0), (0.6, 0.6, -1.0), -0.2),     # outside: 1 - u - v = -0.2
        ((0.2, 0.2, 1.0), (0.2, 0.2, 0.5), -1.0),      # stops short: t = 2, 1 - t = -1
        ((0.2, 0.2, -0.5), (0.2, 0.2, -1.0), -1.0),    # starts beyond: t = -1
        ((0.2, 0.2, 0.9), (0.2, 0.2, -0.1), 0.1),      # crossing at t = 0.9
    ]
    for o, y, want in cases:
        oo, yy = _seg(o, y)
        m, ang = segment_triangle(oo, yy - oo, v0, v1, v2)
        assert abs(m[0, 0] - want) < 1e-12, (o, y, m)
        V, amb = triangle_visibility(oo, yy, UNIT)
        assert V[0] == (0.0 if want > 0 else 1.0) and not amb[0]
    # parallel to the plane: never a hit
    oo, yy = _seg((0.2, 0.2, 0.5), (0.4, 0.1, 0.5))
    m, _ = segment_triangle(oo, yy - oo, v0, v1, v2)
    assert m[0, 0] == -np.inf
    assert triangle_visibility(oo, yy, UNIT)[0][0] == 1.0


def test_triangle_winding_and_direction_do_not_matter():
    flipped = UNIT[:, [0, 1, 2, 6, 7, 8, 3, 4, 5]]
    oo, yy = _seg((0.2, 0.2, 1.0), (0.2, 0.2, -1.0))
    for tri in (UNIT, flipped):
        assert triangle_visibility(oo, yy, tri)[0][0] == 0.0
        assert triangle_visibility(yy, oo, tri)[0][0] == 0.0


def test_triangle_ambiguity_near_an_edge():
    # a segment grazing the edge u = 0 within the margin is flagged, and one
    # clearly inside or outside is not
    for x, flagged in ((0.5 * AMBIG_TRI, True), (-0.5 * AMBIG_TRI, True), (0.01, False), (-0.01, False)):
        oo, yy = _seg((x, 0.3, 1.0), (x, 0.3, -1.0))
        _, amb = triangle_visibility(oo, yy, UNIT)
        assert bool(amb[0]) == flagged, x


def _same_side_visible(o, y, tri):
    """Independent check: the crossing with the plane by the plane equation,
    then the point-in-triangle test by the signs of three cross products."""
    v0, v1, v2 = tri[0:3], tri[3:6], tri[6:9]
    n = np.cross(v1 - v0, v2 - v0)
    D = y - o
    den = n @ D
    if den == 0.0:
        return True
    t = n @ (v0 - o) / den
    if not (0.0 < t < 1.0):
        return True
    p = o + t * D
    c0 = np.cross(v1 - v0, p - v0) @ n
    c1 = np.cross(v2 - v1, p - v1) @ n
    c2 = np.cross(v0 - v2, p - v2) @ n
    inside = (c0 >= 0 and c1 >= 0 and c2 >= 0) or (c0 <= 0 and c1 <= 0 and c2 <= 0)
    return not inside


def test_triangle_visibility_against_an_independent_form():
    rng = np.random.default_rng(12)
    E = 3000
    tri = rng.uniform(-1.0, 1.0, (E, 9))
    o = rng.uniform(-1.5, 1.5, (E, 3))
    y = rng.uniform(-1.5, 1.5, (E, 3))
    blocked = 0
    for k in range(E):
        V, amb = triangle_visibility(o[k:k + 1], y[k:k + 1], tri[k:k + 1])
        if amb[0]:
            continue
        want = _same_side_visible(o[k], y[k], tri[k])
        assert V[0] == (1.0 if want else 0.0), k
        blocked += V[0] == 0.0
    assert 100 < blocked < E - 100      # both outcomes are exercised


def test_entries_with_triangle_occluders():
    # a point under a horizontal triangle, a light above it: blocked; moved
    # aside, the same pair is lit with the closed-form value
    tri = np.array([[-1.0, -1.0, 0.5, 2.0, -1.0, 0.5, -1.0, 2.0, 0.5]])
    x = np.array([[0.0, 0.0, 0.0], [3.0, 3.0, 0.0]])
    nx = np.array([[0.0, 0.0, 1.0]] * 2)
    y = x + np.array([0.0, 0.0, 1.0])
    ny = np.array([[0.0, 0.0, -1.0]] * 2)
    kd = np.full((2, 3), 0.5)
    A, amb, lit = entries(x, nx, kd, np.zeros(2), np.ones(2), np.array([[0, 0, 1.0]] * 2), y, ny,
                          np.ones((2, 3)), {"tri": tri})
    assert lit.all() and not amb.any()
    assert (A[0] == 0.0).all()
    np.testing.assert_allclose(A[1], 0.5 / np.pi * 1.0 * 1.0 / 1.0, rtol=1e-12)
