"""The batching configuration at full size on the GPU: a 1920x1080 image cut
into 1,024 slices of log-uniform rows [64, 4096] (Morton runs), per-slice cuts
of log-uniform size [256, 2048] from 300,000 VPLs, ranks 4, 8, 16 and 32 drawn
per slice, 2.5% + 2.5% sampling, the completion stopping on its tolerance
(at most 100 iterations): the launch configuration the benchmark times for
this workload.

Checked through properties of every slice and, for the smallest slice of
every (rank, completion kernel) pair, stage by stage (pass-1 indices
bit-exact, entries within the per-entry bound, weights and pass-2 indices
bit-exact given the GPU's statistics) and through the oracle's completion of
the GPU's own samples for the GPU's iteration count (1e-3 pixel RMSE)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import check_scene_indices, entries_out_of_tol, keys_to_ij, log  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle.sampling import pass1, pass2, weights_from_g  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene  # noqa: E402

SEED = 21
PPM = 25000


@pytest.fixture(scope="module")
def batch():
    log("batch config: building the scene (1,024 slices, 300,000 VPLs)")
    sc = make_scene("batch", SEED)
    check_scene_indices(sc)
    dev = torch.device("cuda", 0)
    prm = api.default_params(seed=SEED, pass1_ppm=PPM, pass2_ppm=PPM)
    ctx = api.Context(0)
    ctx.set_occluders(sc.spheres)
    ds = api.DeviceScene(sc, dev)
    plan = api.Plan(sc, prm)
    log(f"batch config: {sc.n_slices} slices, workspace {plan.workspace_bytes / 1e9:.1f} GB")
    ws = api.workspace(plan, dev)
    rad = api.render(ctx, plan, ds, prm, ws)
    torch.cuda.synchronize()
    log("batch config: rendered")
    info = [plan.slice_info(s) for s in range(sc.n_slices)]
    out = dict(sc=sc, plan=plan, ws=ws, ctx=ctx, info=info, stats=api.read_stats(ctx, plan, ws),
               radiance=rad.double().cpu().numpy())
    yield out
    del ws
    torch.cuda.empty_cache()


def region(fr, name, dtype, a, n, width=1):
    v = api.region_view(fr["plan"], fr["ws"], name, dtype)
    return v[width * a: width * (a + n)].cpu().numpy()


def samples(fr, s):
    info = fr["info"][s]
    n2 = int(fr["stats"]["n2"][s])
    k1 = region(fr, "OMEGA1", torch.int32, info["off1"], info["N1"])
    k2 = region(fr, "OMEGA2", torch.int32, info["off2"], n2)
    v1 = region(fr, "VAL1", torch.float32, info["off1"], info["N1"], 3).reshape(-1, 3)
    v2 = region(fr, "VAL2", torch.float32, info["off2"], n2, 3).reshape(-1, 3)
    return k1, k2, v1, v2


def strata(fr):
    """The smallest slice of every (rank, kernel) pair present."""
    info = fr["info"]
    best = {}
    for s in range(len(info)):
        key = (info[s]["q"], "ell" if info[s]["adm_in_lds"] else "global")
        if key not in best or (info[s]["m"] * info[s]["n"], s) < (info[best[key]]["m"] * info[best[key]]["n"], best[key]):
            best[key] = s
    return dict(sorted(best.items()))


def test_batch_every_slice(batch):
    sc, info, st = batch["sc"], batch["info"], batch["stats"]
    assert np.isfinite(batch["radiance"]).all()
    q = np.array([i["q"] for i in info])
    assert set(q.tolist()) == {4, 8, 16, 32}
    kinds = {("ell" if i["adm_in_lds"] else "global") for i in info}
    assert kinds == {"ell", "global"}
    assert ((st["iters"] >= 1) & (st["iters"] <= 100)).all()
    n2 = st["n2"].astype(np.int64)
    N2 = np.array([i["N2"] for i in info])
    short = (st["flags"] & 4) != 0
    assert np.array_equal(n2[~short], N2[~short])
    assert (n2[short] < N2[short]).all()
    for s in range(0, sc.n_slices, 16):
        k1, k2, _, _ = samples(batch, s)
        i1, j1 = keys_to_ij(k1)
        i2, j2 = keys_to_ij(k2)
        mm, nn = info[s]["m"], info[s]["n"]
        e = np.concatenate([i1 * nn + j1, i2 * nn + j2])
        assert i1.max() < mm and j1.max() < nn and (i2.size == 0 or (i2.max() < mm and j2.max() < nn))
        assert np.unique(e).shape[0] == e.shape[0]
    outside = np.setdiff1d(np.arange(sc.m), sc.pt_ids)
    assert (batch["radiance"][outside] == 0).all()
    log(f"batch config: {int(short.sum())} slices short in pass 2; iterations {int(st['iters'].min())}-"
        f"{int(st['iters'].max())}; strata {list(strata(batch))}")


def test_batch_strata_stage_parity(batch):
    sc, info = batch["sc"], batch["info"]
    lights = orender.cluster_lights(sc, SEED)
    p = orender.Params(seed=SEED, pass1_ppm=PPM, pass2_ppm=PPM)
    for key, s in strata(batch).items():
        m, n = info[s]["m"], info[s]["n"]
        log(f"batch slice {s} {key} (m={m}, n={n}): pass 1, entries, weights, pass 2")
        k1, k2, v1, _ = samples(batch, s)
        gi, gj = keys_to_ij(k1)
        i1, j1 = pass1(SEED, s, m, n, PPM)
        assert np.array_equal(gi, i1) and np.array_equal(gj, j1)
        sel = np.random.default_rng(s).choice(i1.shape[0], min(2000, i1.shape[0]), replace=False)
        o, amb, _ = orender.eval_entries(sc, lights, sc.slice_rows(s)[gi[sel]], sc.slice_cols(s)[gj[sel]], p)
        assert not entries_out_of_tol(v1[sel], o, amb).any()
        a = info[s]["off_col"]
        gmin = region(batch, "COLMIN", torch.float32, a, n)
        gmax = region(batch, "COLMAX", torch.float32, a, n)
        cnt = region(batch, "COLCNT", torch.int32, a, n)
        g32 = np.where(cnt > 0, (gmax - gmin).astype(np.float32), np.float32(0))
        w = region(batch, "WEIGHTS", torch.int32, a, n).astype(np.uint64)
        assert np.array_equal(w, weights_from_g(g32.astype(np.float64)))
        taken = np.zeros(m * n, bool)
        taken[gi * n + gj] = True
        i2, j2, short = pass2(SEED, s, m, n, info[s]["N1"], PPM, w, taken)
        gi2, gj2 = keys_to_ij(k2)
        assert np.array_equal(gi2, i2) and np.array_equal(gj2, j2)
        assert bool(short) == bool(batch["stats"]["flags"][s] & 4)


def test_batch_strata_completion_on_the_gpu_samples(batch):
    """The oracle's completion of the GPU's own samples, run for the number of
    iterations the GPU's tolerance test stopped at, against the GPU's
    radiance: every (rank, kernel) pair."""
    sc, info, st = batch["sc"], batch["info"], batch["stats"]
    for key, s in strata(batch).items():
        m, n, q = info[s]["m"], info[s]["n"], info[s]["q"]
        it = int(st["iters"][s])
        p = orender.Params(seed=SEED, pass1_ppm=PPM, pass2_ppm=PPM, max_iter=max(it, 1), fixed_iters=True)
        k1, k2, v1, v2 = samples(batch, s)
        ii, jj = keys_to_ij(np.concatenate([k1, k2]))
        A = np.concatenate([v1, v2]).astype(np.float64)
        I, *_ = orender.complete_and_render(m, n, q, ii, jj, A, SEED, s, p)
        rel = orender.relative_rmse(batch["radiance"][sc.slice_rows(s)], I)
        log(f"batch slice {s} {key} (m={m}, n={n}, {it} iterations): pixel RMSE vs oracle {rel:.2e}")
        assert rel <= 1e-3, f"slice {s} {key}: {rel:.2e}"
