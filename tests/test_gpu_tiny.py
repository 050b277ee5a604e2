"""Parity of the HIP path with the FP64 oracle on the tiny workload
(64x64 points, 32 spheres, 1,024 singleton clusters, 16 slices of 256,
rank 8, 5% + 5%), stage by stage and end to end, through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import keys_to_ij, log, omega_of, run_frame, entries_out_of_tol  # noqa: E402
from oracle import adm as oadm  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle.cluster import cluster_table  # noqa: E402
from oracle.philox import philox4x64_vec  # noqa: E402
from oracle.sampling import pass1, pass2, weights_from_g  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene  # noqa: E402

SEED = 1
ITERS = 100


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
    return make_scene("tiny", SEED)


@pytest.fixture(scope="module")
def run(scene):
    return run_frame(scene, gpu_params(), label="tiny")


@pytest.fixture(scope="module")
def lights(scene):
    return orender.cluster_lights(scene, SEED)


def slice_view(run, name, s, width=1):
    info = run["info"][s]
    r = run["r"][name]
    if name in ("OMEGA1", "VAL1"):
        a, n = info["off1"], info["N1"]
    elif name in ("OMEGA2", "VAL2"):
        a, n = info["off2"], int(run["stats"]["n2"][s])
    elif name in ("WEIGHTS", "COLMIN", "COLMAX", "COLCNT"):
        a, n = info["off_col"], info["n"]
    elif name == "ROW_PTR":
        a, n = info["off_row"], info["m"] + 1
    elif name == "COL_PTR":
        a, n = info["off_colptr"], info["n"] + 1
    elif name in ("CSR_COL", "CSC_ROW", "CSR_VAL", "CSC_VAL"):
        a, n = info["off_omega"], info["N1"] + int(run["stats"]["n2"][s])
    elif name == "X":
        a, n = info["off_x"], info["m"] * info["q_pad"]
    elif name == "Y":
        a, n = info["off_y"], 3 * info["n"] * info["q_pad"]
    else:
        raise KeyError(name)
    return r[width * a: width * (a + n)]


def test_philox_bit_exact(run):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, (4096, 4), dtype=np.int64)
    for key in [(0, 0), (1, 7), (2**63 + 5, 123456789)]:
        out = api.philox4x64(run["ctx"], key[0], key[1], torch.as_tensor(ctr).cuda()).cpu().numpy()
        want = philox4x64_vec(key[0], key[1], *(ctr[:, k].astype(np.uint64) for k in range(4)))
        for k in range(4):
            assert np.array_equal(out[:, k].astype(np.uint64), want[k])


def test_cluster_table_bit_exact(run, scene):
    rep, inten, lo, hi = cluster_table(scene.vpls, scene.cut_offsets, scene.cut_members, SEED)
    assert np.array_equal(slice_of_region(run, "REP"), rep)
    L = run["r"]["LIGHTS"].reshape(9, -1)
    assert np.array_equal(L[6:9].T.view(np.uint32), inten.view(np.uint32))
    assert np.array_equal(L[0], scene.vpls["x"][rep])


def slice_of_region(run, name):
    return run["r"][name][: run["plan"].n_clusters]


def test_cluster_table_clustered_cut():
    """A cut of multi-member clusters: representative ids and FP32-rounded
    FP64 intensity sums are bit-exact."""
    import dataclasses
    from scenegen import CONFIGS
    cfg = dataclasses.replace(CONFIGS["mid"], width=32, height=32, n_slices=4, n_vpls=4096, n_clusters=300)
    sc = make_scene(cfg, 5)
    ds = api.DeviceScene(sc, torch.device("cuda", 0))
    ctx = api.Context(0)
    for seed in (3, 4):
        rep, L, bbox = api.cluster_table(ctx, ds, seed)
        orep, ointen, olo, ohi = cluster_table(sc.vpls, sc.cut_offsets, sc.cut_members, seed)
        assert np.array_equal(rep.cpu().numpy(), orep)
        L = L.cpu().numpy()
        assert np.array_equal(L[6:9].T.view(np.uint32), ointen.view(np.uint32))
        assert np.array_equal(bbox.cpu().numpy()[:3].T, olo) and np.array_equal(bbox.cpu().numpy()[3:].T, ohi)


def test_pass1_bit_exact(run, scene):
    for s in range(scene.n_slices):
        info = run["info"][s]
        i1, j1 = pass1(SEED, s, info["m"], info["n"], 50000)
        gi, gj = keys_to_ij(slice_view(run, "OMEGA1", s))
        assert np.array_equal(gi, i1) and np.array_equal(gj, j1), f"slice {s}"


def test_first_pass_entries(run, scene, lights):
    p = oracle_params()
    total_amb = 0
    for s in range(scene.n_slices):
        gi, gj = keys_to_ij(slice_view(run, "OMEGA1", s))
        o, amb, _ = orender.eval_entries(scene, lights, scene.slice_rows(s)[gi], scene.slice_cols(s)[gj], p)
        g = slice_view(run, "VAL1", s, 3).reshape(-1, 3)
        bad = entries_out_of_tol(g, o, amb)
        total_amb += int(amb.sum())
        assert not bad.any(), f"slice {s}: {int(bad.any(axis=1).sum())} entries out of tolerance"
    log(f"first-pass ambiguous-visibility entries excluded: {total_amb}")


def test_column_stats_and_weights(run, scene):
    mismatch = 0
    total = 0
    worst = 0.0
    for s in range(scene.n_slices):
        n = run["info"][s]["n"]
        _, gj = keys_to_ij(slice_view(run, "OMEGA1", s))
        v = slice_view(run, "VAL1", s, 3).reshape(-1, 3).astype(np.float32)
        t = (v[:, 0] + v[:, 1]) + v[:, 2]
        cnt = np.bincount(gj, minlength=n)
        assert np.array_equal(slice_view(run, "COLCNT", s), cnt)
        mx = np.zeros(n, np.float32)
        mn = np.full(n, np.inf, np.float32)
        np.maximum.at(mx, gj, t)
        np.minimum.at(mn, gj, t)
        gmin, gmax = slice_view(run, "COLMIN", s), slice_view(run, "COLMAX", s)
        seen = cnt > 0
        assert np.array_equal(gmin[seen], mn[seen]) and np.array_equal(gmax[seen], mx[seen])
        g32 = np.where(seen, (gmax - gmin).astype(np.float32), np.float32(0))
        w_same_precision = weights_from_g(g32.astype(np.float64))
        w_gpu = slice_view(run, "WEIGHTS", s).astype(np.uint64)
        assert np.array_equal(w_gpu, w_same_precision), f"slice {s}"
        # against the oracle's own FP64 entries: reported, not required to match
        r = orender.render_slice(scene, orender.cluster_lights(scene, SEED), s, oracle_params(max_iter=0), keep=True)
        mismatch += int((r["w"] != w_gpu).sum())
        total += n
        # w resolves g to 2^-24 of its maximum, finer than FP32 entries: the
        # quantised pdf may differ by FP32 rounding of g, i.e. ~1e-6 of max g
        worst = max(worst, float(np.abs(r["w"].astype(np.float64) - w_gpu.astype(np.float64)).max()) / 2 ** 24)
    log(f"weights differing from the FP64-entry oracle: {mismatch} of {total}; largest difference "
        f"{worst:.2e} of the maximum weight")
    assert worst <= 1e-5


def test_pass2_bit_exact_given_weights(run, scene):
    for s in range(scene.n_slices):
        info = run["info"][s]
        m, n = info["m"], info["n"]
        gi1, gj1 = keys_to_ij(slice_view(run, "OMEGA1", s))
        taken = np.zeros(m * n, bool)
        taken[gi1 * n + gj1] = True
        w = slice_view(run, "WEIGHTS", s).astype(np.uint64)
        i2, j2, short = pass2(SEED, s, m, n, info["N1"], 50000, w, taken)
        gi2, gj2 = keys_to_ij(slice_view(run, "OMEGA2", s))
        assert np.array_equal(gi2, i2) and np.array_equal(gj2, j2), f"slice {s}"
        assert bool(run["stats"]["flags"][s] & 4) == short


def test_column_pointers_and_distinct_samples(run, scene):
    """Every slice here is completed from its ELL copy (checked through the
    completion itself); the column pointers cover Omega = Omega1 u Omega2, whose
    entries are distinct."""
    for s in range(scene.n_slices):
        info = run["info"][s]
        m, n = info["m"], info["n"]
        assert info["adm_in_lds"] == 1
        i, j, _ = omega_of(run, s)
        assert np.unique(i * n + j).shape[0] == i.shape[0]
        cp = np.concatenate([[0], np.cumsum(np.bincount(j, minlength=n))])
        assert np.array_equal(slice_view(run, "COL_PTR", s), cp)


def test_initial_factors_bit_exact(scene):
    r0 = run_frame(scene, gpu_params(max_iter=0), label="tiny max_iter=0")
    for s in (0, 7, 15):
        info = r0["info"][s]
        m, n, q = info["m"], info["n"], info["q"]
        X0, Y0 = oadm.init_factors(SEED, s, m, 3 * n, q)
        gX = slice_view(r0, "X", s).reshape(m, q)
        gY = slice_view(r0, "Y", s).reshape(n, 3, q)
        assert np.array_equal(gX, X0.astype(np.float32))
        Yo = Y0.reshape(q, 3, n).transpose(2, 1, 0)
        assert np.array_equal(gY, Yo.astype(np.float32))


def adm_on_gpu_samples(run, s, iters=ITERS):
    info = run["info"][s]
    m, n, q = info["m"], info["n"], info["q"]
    ii, jj, A = omega_of(run, s)
    A = A.astype(np.float64)
    p = oracle_params(max_iter=iters)
    return orender.complete_and_render(m, n, q, ii, jj, A, SEED, s, p)


def test_adm_and_reduce_match_oracle_on_identical_samples(run, scene):
    worst = 0.0
    for s in range(scene.n_slices):
        I, iters, err, flags, fac = adm_on_gpu_samples(run, s)
        g = run["radiance"][scene.slice_rows(s)]
        rel = orender.relative_rmse(g, I)
        worst = max(worst, rel)
        assert rel <= 1e-3, f"slice {s}: pixel relative RMSE {rel:.2e}"
        assert abs(float(run["r"]["SLICE_SCALE"][s]) - fac[2]) <= 1e-6 * fac[2]
        assert abs(float(run["stats"]["resid"][s]) - err) <= 1e-3 * err + 1e-6
    log(f"ADM + reduce worst slice pixel RMSE vs oracle: {worst:.2e}")


def test_end_to_end_against_oracle(run, scene):
    """The whole frame through the oracle (second pass given the GPU's
    quantised weights, the one place where FP32 decides an integer)."""
    wo = {s: slice_view(run, "WEIGHTS", s).astype(np.uint64) for s in range(scene.n_slices)}
    I, per = orender.render(scene, oracle_params(), weights_override=wo)
    rel = orender.relative_rmse(run["radiance"], I)
    log(f"end-to-end pixel RMSE vs oracle: {rel:.2e}; ambiguous entries "
        f"{sum(r['n_ambiguous'] for r in per)}")
    assert rel <= 1e-3


def test_tolerance_mode_reports_iterations(scene):
    r = run_frame(scene, gpu_params(fixed_iters=False, tol=0.5, max_iter=100), regions=False, label="tol 0.5")
    st = r["stats"]
    assert (st["iters"] < 100).all() and (st["resid"] < 0.5).all()
    r2 = run_frame(scene, gpu_params(fixed_iters=False, tol=1e-9, max_iter=3), regions=False, label="tol 1e-9")
    assert (r2["stats"]["iters"] == 3).all() and (r2["stats"]["flags"] & 2).all()


def test_eval_pairs_random(run, scene, lights):
    rng = np.random.default_rng(4)
    n = 20000
    pid = rng.integers(0, scene.m, n).astype(np.int32)
    lid = rng.integers(0, scene.n, n).astype(np.int32)
    ds = run["ds"]
    out = api.eval_pairs(run["ctx"], ds, ds.vpl, torch.as_tensor(pid).cuda(), torch.as_tensor(lid).cuda(),
                         gpu_params()).cpu().numpy()
    from oracle.shading import entries, point_arrays
    V = scene.vpls
    x, nn, kd, ks, pe, wo = point_arrays(scene.points, pid)
    pos = np.stack([V["x"], V["y"], V["z"]], 1)[lid]
    nrm = np.stack([V["nx"], V["ny"], V["nz"]], 1)[lid]
    inten = np.stack([V["ir"], V["ig"], V["ib"]], 1)[lid]
    o, amb, lit = entries(x, nn, kd, ks, pe, wo, pos, nrm, inten, scene.spheres)
    assert not entries_out_of_tol(out, o, amb).any()
    assert lit.sum() > 1000 and (o[lit].sum(1) == 0).sum() > 100      # shadows present


def test_brute_force_matches_oracle(run, scene):
    rng = np.random.default_rng(2)
    pid = rng.choice(scene.m, 96, replace=False).astype(np.int32)
    ds = run["ds"]
    g = api.brute_force(run["ctx"], ds, ds.vpl, gpu_params(), point_ids=torch.as_tensor(pid).cuda()).cpu().numpy()
    o = orender.brute_force(scene, oracle_params(), point_ids=pid)
    # pixels one of whose 1,024 entries has a visibility within 1e-5 of flipping
    # may differ by a whole entry; every other pixel holds to 1e-4
    from oracle.shading import entries, point_arrays
    V = scene.vpls
    pr = np.repeat(pid, scene.n)
    lj = np.tile(np.arange(scene.n), pid.shape[0])
    x, nn, kd, ks, pe, wo = point_arrays(scene.points, pr)
    pos = np.stack([V["x"], V["y"], V["z"]], 1)[lj]
    nrm = np.stack([V["nx"], V["ny"], V["nz"]], 1)[lj]
    inten = np.stack([V["ir"], V["ig"], V["ib"]], 1)[lj]
    _, amb, _ = entries(x, nn, kd, ks, pe, wo, pos, nrm, inten, scene.spheres)
    clear = ~amb.reshape(pid.shape[0], scene.n).any(axis=1)
    rel = np.abs(g - o) / np.maximum(np.abs(o), 1e-12)
    log(f"brute force: {clear.sum()} of {pid.shape[0]} pixels without an ambiguous entry, "
        f"max relative error there {rel[clear].max():.2e}")
    assert clear.sum() >= 80
    assert rel[clear].max() <= 1e-4


def test_full_sampling_takes_the_rest_in_row_major_order(scene):
    """100% sampling (5% uniform + 95%): the second pass is every entry the
    first pass left, in row-major order, bit for bit; the completion of the
    fully observed slices matches the oracle's (30 fixed iterations)."""
    prm = gpu_params(pass1_ppm=50000, pass2_ppm=950000, max_iter=30)
    r = run_frame(scene, prm, label="tiny at 100%")
    for s in range(scene.n_slices):
        info = r["info"][s]
        m, n = info["m"], info["n"]
        assert info["N1"] + info["N2"] == m * n
        assert int(r["stats"]["n2"][s]) == info["N2"] and not (r["stats"]["flags"][s] & 4)
        i1, j1 = pass1(SEED, s, m, n, 50000)
        taken = np.zeros(m * n, bool)
        taken[i1 * n + j1] = True
        i2, j2, short = pass2(SEED, s, m, n, i1.shape[0], 950000, np.ones(n, np.uint64), taken)
        gi, gj = keys_to_ij(slice_view(r, "OMEGA2", s))
        assert not short and np.array_equal(gi, i2) and np.array_equal(gj, j2), f"slice {s}"
    slices = [0, 9]
    I, _ = orender.render(scene, oracle_params(pass1_ppm=50000, pass2_ppm=950000, max_iter=30), slices=slices)
    for s in slices:
        pid = scene.slice_rows(s)
        rel = orender.relative_rmse(r["radiance"][pid], I[pid])
        log(f"100% sampling, slice {s}: pixel RMSE vs oracle {rel:.2e}")
        assert rel <= 1e-3


def test_all_zero_slice_is_flagged_and_black(scene):
    """Every VPL turned to face up (away from every surface point below it):
    every entry is 0, so every slice is flagged VPLMC_SLICE_ALL_ZERO and its
    radiance is exactly 0 (the completion is skipped, Appendix A has nothing
    to fit)."""
    import dataclasses
    v = dict(scene.vpls)
    v["nx"] = np.zeros_like(v["nx"])
    v["ny"] = np.zeros_like(v["ny"])
    v["nz"] = np.ones_like(v["nz"])
    sc = dataclasses.replace(scene, vpls=v)
    r = run_frame(sc, gpu_params(max_iter=10), label="all-zero")
    assert (r["stats"]["flags"] & 1).all()
    assert not np.any(r["radiance"])
    assert not np.any(r["r"]["VAL1"]) and not np.any(r["r"]["VAL2"])


def test_ranks_between_the_kernel_ranks(scene):
    """Ranks 1, 2, 3, 5, 7, 12 and 20 (padded to the kernels' 4, 8, 16, 32 with
    zero components): the oracle's rank-q ADM on the GPU's samples, 1e-3;
    rank 20 on a 256-row slice runs the global-memory kernel (rank 32), the
    others the LDS-resident one."""
    from scenegen import scene_sample
    ranks = [1, 2, 3, 5, 7, 12, 20]
    sub = scene_sample(scene, list(range(len(ranks))))
    sub.rank = np.asarray(ranks, np.int32)
    r = run_frame(sub, gpu_params(max_iter=40), label="ranks 1-20")
    worst = 0.0
    for s, q in enumerate(ranks):
        info = r["info"][s]
        assert info["q"] == q and info["q_pad"] == (4 if q <= 4 else 8 if q <= 8 else 16 if q <= 16 else 32)
        ii, jj, A = omega_of(r, s)
        I, *_ = orender.complete_and_render(info["m"], info["n"], q, ii, jj, A.astype(np.float64), SEED, s,
                                            oracle_params(max_iter=40))
        rel = orender.relative_rmse(r["radiance"][sub.slice_rows(s)], I)
        worst = max(worst, rel)
        assert rel <= 1e-3, f"rank {q}: pixel RMSE {rel:.2e}"
        # the padded components of X stay exactly zero
        X = r["r"]["X"][info["off_x"]: info["off_x"] + info["m"] * info["q_pad"]].reshape(info["m"], -1)
        assert not X[:, q:].any()
    log(f"ranks {ranks}: worst pixel RMSE vs oracle {worst:.2e}")
