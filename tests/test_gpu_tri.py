"""The triangle workload on the GPU (Sec. 6: visibility rays through an
SBVH over triangles): 64x64 points on 32 icospheres of 320 faces and a
ground plane (10,242 triangles), 1,024 instant-radiosity VPLs as singleton
clusters, 16 slices, rank 8, 5% + 5%.  Against the FP64 oracle, which
decides visibility by brute force over every triangle: random (point, VPL)
entries, every stage of three slices (pass 1 bit-exact, entries, the
completion of the GPU's own samples) and brute-force pixel sums; ambiguous
entries (a triangle within 1e-4 of flipping the outcome in barycentric or
segment parameters) are excluded and counted."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import entries_out_of_tol, keys_to_ij, log, omega_of, run_frame  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle.sampling import pass1  # noqa: E402
from oracle.shading import entries, point_arrays  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene  # noqa: E402

SEED = 1
ITERS = 30


def gpu_params(**kw):
    base = dict(seed=SEED, pass1_ppm=50000, pass2_ppm=50000, max_iter=ITERS, fixed_iters=True)
    base.update(kw)
    return api.default_params(**base)


def oracle_params(**kw):
    base = dict(seed=SEED, pass1_ppm=50000, pass2_ppm=50000, max_iter=ITERS, fixed_iters=True)
    base.update(kw)
    return orender.Params(**base)


@pytest.fixture(scope="module")
def scene():
    sc = make_scene("tri", SEED)
    log(f"tri scene: {sc.spheres['tri'].shape[0]} triangles, {sc.n} VPLs")
    return sc


@pytest.fixture(scope="module")
def run(scene):
    return run_frame(scene, gpu_params(), label="tri")


def _pairs(scene, pid, lid):
    V = scene.vpls
    x, nn, kd, ks, pe, wo = point_arrays(scene.points, pid)
    pos = np.stack([V["x"], V["y"], V["z"]], 1)[lid]
    nrm = np.stack([V["nx"], V["ny"], V["nz"]], 1)[lid]
    inten = np.stack([V["ir"], V["ig"], V["ib"]], 1)[lid]
    return entries(x, nn, kd, ks, pe, wo, pos, nrm, inten, scene.spheres)


def test_eval_pairs_random(run, scene):
    rng = np.random.default_rng(4)
    n = 20000
    pid = rng.integers(0, scene.m, n).astype(np.int32)
    lid = rng.integers(0, scene.n, n).astype(np.int32)
    ds = run["ds"]
    out = api.eval_pairs(run["ctx"], ds, ds.vpl, torch.as_tensor(pid).cuda(), torch.as_tensor(lid).cuda(),
                         gpu_params()).cpu().numpy()
    o, amb, lit = _pairs(scene, pid, lid)
    bad = entries_out_of_tol(out, o, amb)
    log(f"tri pairs: {int(lit.sum())} lit, {int((o[lit].sum(1) == 0).sum())} of them shadowed, "
        f"{int(amb.sum())} ambiguous")
    assert not bad.any(), f"{int(bad.any(axis=1).sum())} entries out of tolerance"
    assert lit.sum() > 1000 and (o[lit].sum(1) == 0).sum() > 100       # shadows present


def test_slices_stage_by_stage(run, scene):
    lights = orender.cluster_lights(scene, SEED)
    p = oracle_params()
    for s in (0, 7, 15):
        info = run["info"][s]
        m, n, q = info["m"], info["n"], info["q"]
        k1 = run["r"]["OMEGA1"][info["off1"]: info["off1"] + info["N1"]]
        gi, gj = keys_to_ij(k1)
        i1, j1 = pass1(SEED, s, m, n, 50000)
        assert np.array_equal(gi, i1) and np.array_equal(gj, j1), f"slice {s}"
        ii, jj, A = omega_of(run, s)
        o, amb, _ = orender.eval_entries(scene, lights, scene.slice_rows(s)[ii], scene.slice_cols(s)[jj], p)
        assert not entries_out_of_tol(A, o, amb).any(), f"slice {s}"
        order = np.argsort(ii * n + jj, kind="stable")
        I, *_ = orender.complete_and_render(m, n, q, ii[order], jj[order], A[order].astype(np.float64), SEED, s, p)
        rel = orender.relative_rmse(run["radiance"][scene.slice_rows(s)], I)
        log(f"tri slice {s}: {int(amb.sum())} ambiguous entries; ADM on the GPU's samples {rel:.2e}")
        assert rel <= 1e-3


def test_brute_force_matches_oracle(run, scene):
    rng = np.random.default_rng(2)
    pid = rng.choice(scene.m, 32, replace=False).astype(np.int32)
    ds = run["ds"]
    g = api.brute_force(run["ctx"], ds, ds.vpl, gpu_params(), point_ids=torch.as_tensor(pid).cuda()).cpu().numpy()
    o = orender.brute_force(scene, oracle_params(), point_ids=pid)
    pr = np.repeat(pid, scene.n)
    lj = np.tile(np.arange(scene.n), pid.shape[0])
    _, amb, _ = _pairs(scene, pr, lj)
    clear = ~amb.reshape(pid.shape[0], scene.n).any(axis=1)
    rel = np.abs(g - o) / np.maximum(np.abs(o), 1e-12)
    log(f"tri brute force: {clear.sum()} of {pid.shape[0]} pixels without an ambiguous entry, "
        f"max relative error there {rel[clear].max():.2e}")
    assert clear.sum() >= 24
    assert rel[clear].max() <= 1e-4


def test_triangles_replace_spheres_and_back(scene):
    """set_occluders with triangles, then with no occluders: an entry that a
    triangle shadows is dark, then lit."""
    ctx = api.Context(0)
    ds = api.DeviceScene(scene, torch.device("cuda", 0))
    rng = np.random.default_rng(9)
    pid = rng.integers(0, scene.m, 4000).astype(np.int32)
    lid = rng.integers(0, scene.n, 4000).astype(np.int32)
    o, amb, lit = _pairs(scene, pid, lid)
    shadowed = lit & ~amb & (o.sum(1) == 0)
    assert shadowed.sum() > 20
    ctx.set_occluders(scene.spheres)
    a = api.eval_pairs(ctx, ds, ds.vpl, torch.as_tensor(pid).cuda(), torch.as_tensor(lid).cuda(),
                       gpu_params()).cpu().numpy()
    assert (a[shadowed] == 0).all()
    ctx.set_occluders({"tri": np.zeros((0, 9), np.float32)})
    b = api.eval_pairs(ctx, ds, ds.vpl, torch.as_tensor(pid).cuda(), torch.as_tensor(lid).cuda(),
                       gpu_params()).cpu().numpy()
    assert (b[shadowed].sum(1) > 0).all()


def test_trimid_entries_sampled():
    """The 512x512 triangle workload at full size (163,842 triangles, an SBVH
    of ~213,000 nodes with spatial splits, 65,536 instant-radiosity VPLs):
    3,000 random (point, VPL) entries against the oracle's brute force over
    every triangle."""
    sc = make_scene("trimid", 11)
    log(f"trimid: {sc.spheres['tri'].shape[0]} triangles, {sc.n} VPLs")
    ctx = api.Context(0)
    ctx.set_occluders(sc.spheres)
    ds = api.DeviceScene(sc, torch.device("cuda", 0))
    rng = np.random.default_rng(8)
    n = 3000
    pid = rng.integers(0, sc.m, n).astype(np.int32)
    lid = rng.integers(0, sc.n, n).astype(np.int32)
    out = api.eval_pairs(ctx, ds, ds.vpl, torch.as_tensor(pid).cuda(), torch.as_tensor(lid).cuda(),
                         gpu_params()).cpu().numpy()
    o, amb, lit = _pairs(sc, pid, lid)
    bad = entries_out_of_tol(out, o, amb)
    log(f"trimid pairs: {int(lit.sum())} lit, {int((o[lit].sum(1) == 0).sum())} shadowed, {int(amb.sum())} ambiguous")
    assert not bad.any(), f"{int(bad.any(axis=1).sum())} entries out of tolerance"
    assert (o[lit].sum(1) == 0).sum() > 30
