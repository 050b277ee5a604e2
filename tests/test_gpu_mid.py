"""Parity of the HIP path with the FP64 oracle at full size: the mid workload
(512x512 points, 512 spheres, 65,536 VPLs cut to 4,096 clusters, 256 slices
of 1,024, rank 16, 5%) in the configuration the benchmark times, checked on
sampled slices stage by stage and on every slice through properties that hold
at any size; and an uneven batch (row counts, cut sizes and ranks drawn per
slice) that exercises both ADM kernel variants."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import check_csr_csc, keys_to_ij, log, omega_of, run_frame, entries_out_of_tol  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle.sampling import pass1, pass2, weights_from_g  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import CONFIGS, make_scene  # noqa: E402

SEED = 11
PPM = 25000
SAMPLED = (0, 77, 255)


@pytest.fixture(scope="module")
def mid():
    sc = make_scene("mid", SEED)
    prm = api.default_params(seed=SEED, pass1_ppm=PPM, pass2_ppm=PPM)
    return sc, run_frame(sc, prm, label="mid 5%")


def view(run, name, s, width=1):
    info = run["info"][s]
    r = run["r"][name]
    n2 = int(run["stats"]["n2"][s])
    a, n = {"OMEGA1": (info["off1"], info["N1"]), "VAL1": (info["off1"], info["N1"]),
            "OMEGA2": (info["off2"], n2), "VAL2": (info["off2"], n2),
            "WEIGHTS": (info["off_col"], info["n"]), "COLMIN": (info["off_col"], info["n"]),
            "COLMAX": (info["off_col"], info["n"]), "COLCNT": (info["off_col"], info["n"]),
            "ROW_PTR": (info["off_row"], info["m"] + 1), "COL_PTR": (info["off_colptr"], info["n"] + 1),
            "CSR_COL": (info["off_omega"], info["N1"] + n2), "CSR_VAL": (info["off_omega"], info["N1"] + n2),
            "CSC_ROW": (info["off_omega"], info["N1"] + n2), "CSC_VAL": (info["off_omega"], info["N1"] + n2),
            }[name]
    return r[width * a: width * (a + n)]


def test_every_slice_properties(mid):
    sc, run = mid
    st = run["stats"]
    assert np.isfinite(run["radiance"]).all()
    for s in range(sc.n_slices):
        info = run["info"][s]
        m, n = info["m"], info["n"]
        i1, j1 = keys_to_ij(view(run, "OMEGA1", s))
        i2, j2 = keys_to_ij(view(run, "OMEGA2", s))
        e1, e2 = i1 * n + j1, i2 * n + j2
        assert i1.max() < m and j1.max() < n
        assert np.unique(e1).shape[0] == info["N1"]
        assert np.unique(e2).shape[0] == e2.shape[0] == info["N2"]
        assert not np.isin(e2, e1).any()
        assert int(view(run, "COL_PTR", s)[-1]) == info["N1"] + info["N2"]
    assert (st["iters"] == 100).all()
    assert not (st["flags"] & 4).any()


def test_sampled_slices_stage_parity(mid):
    sc, run = mid
    lights = orender.cluster_lights(sc, SEED)
    p = orender.Params(seed=SEED, pass1_ppm=PPM, pass2_ppm=PPM)
    for s in SAMPLED:
        info = run["info"][s]
        m, n = info["m"], info["n"]
        log(f"mid slice {s}: pass 1")
        i1, j1 = pass1(SEED, s, m, n, PPM)
        gi, gj = keys_to_ij(view(run, "OMEGA1", s))
        assert np.array_equal(gi, i1) and np.array_equal(gj, j1)
        log(f"mid slice {s}: entries")
        sel = np.random.default_rng(s).choice(i1.shape[0], 20000, replace=False)
        o, amb, _ = orender.eval_entries(sc, lights, sc.slice_rows(s)[gi[sel]], sc.slice_cols(s)[gj[sel]], p)
        g = view(run, "VAL1", s, 3).reshape(-1, 3)[sel]
        assert not entries_out_of_tol(g, o, amb).any()
        log(f"mid slice {s}: weights and pass 2")
        gmin, gmax, cnt = view(run, "COLMIN", s), view(run, "COLMAX", s), view(run, "COLCNT", s)
        g32 = np.where(cnt > 0, (gmax - gmin).astype(np.float32), np.float32(0))
        w = view(run, "WEIGHTS", s).astype(np.uint64)
        assert np.array_equal(w, weights_from_g(g32.astype(np.float64)))
        taken = np.zeros(m * n, bool)
        taken[gi * n + gj] = True
        i2, j2, short = pass2(SEED, s, m, n, info["N1"], PPM, w, taken)
        gi2, gj2 = keys_to_ij(view(run, "OMEGA2", s))
        assert np.array_equal(gi2, i2) and np.array_equal(gj2, j2) and not short


def test_sampled_slices_adm_parity(mid):
    sc, run = mid
    p = orender.Params(seed=SEED, pass1_ppm=PPM, pass2_ppm=PPM, fixed_iters=True)
    for s in SAMPLED[:2]:
        info = run["info"][s]
        m, n, q = info["m"], info["n"], info["q"]
        log(f"mid slice {s}: oracle ADM on the GPU's samples")
        ii, jj, A = omega_of(run, s)
        A = A.astype(np.float64)
        I, iters, err, flags, fac = orender.complete_and_render(m, n, q, ii, jj, A, SEED, s, p)
        rel = orender.relative_rmse(run["radiance"][sc.slice_rows(s)], I)
        log(f"mid slice {s}: pixel RMSE vs oracle {rel:.2e}")
        assert rel <= 1e-3


# largest per-slice end-to-end bound the sensitivity rule may grant
CEILING = 1e-2

BATCH = dataclasses.replace(CONFIGS["batch"], width=320, height=200, n_spheres=256, n_vpls=8000,
                            batch_slices=24, batch_m=(64, 2048), batch_n=(256, 1024))


@pytest.fixture(scope="module")
def batch():
    sc = make_scene(BATCH, 21)
    prm = api.default_params(seed=21, pass1_ppm=PPM, pass2_ppm=PPM, max_iter=40, fixed_iters=True)
    return sc, run_frame(sc, prm, label="uneven batch")


def test_uneven_batch_against_oracle(batch):
    """Slices of uneven rows, cut sizes and ranks, large slices completing in
    the global-memory ADM kernel and small ones in the LDS one.

    (1) completion parity: the oracle's ADM on the GPU's own samples (same
    FP32 entry values) against the GPU's radiance, 1e-3 pixel RMSE per slice;
    (2) the whole path: the oracle's frame (its own FP64 entries, the GPU's
    weights) against the GPU's frame, 1e-3 over all pixels; per slice the
    bound is 1e-3 or 50 x the oracle's own response to 1e-6 relative noise on
    its entries, whichever is larger: an unconverged low-rank completion can
    amplify input rounding by orders of magnitude, and the entries themselves
    may differ by FP32 rounding of the shading; the bound never exceeds
    CEILING whatever the sensitivity."""
    sc, run = batch
    variants = {"lds" if run["info"][s]["adm_in_lds"] else "global" for s in range(sc.n_slices)}
    log(f"batch ranks {sorted(set(sc.rank.tolist()))}, ADM variants {sorted(variants)}")
    assert variants == {"lds", "global"}
    p = orender.Params(seed=21, pass1_ppm=PPM, pass2_ppm=PPM, max_iter=40, fixed_iters=True)
    # (1) identical samples
    for s in range(sc.n_slices):
        info = run["info"][s]
        m, n, q = info["m"], info["n"], info["q"]
        if not info["adm_in_lds"]:
            check_csr_csc(run, s)       # the global-memory kernel's input orders
        ii, jj, A = omega_of(run, s)
        A = A.astype(np.float64)
        I, *_ = orender.complete_and_render(m, n, q, ii, jj, A, 21, s, p)
        rel = orender.relative_rmse(run["radiance"][sc.slice_rows(s)], I)
        log(f"batch slice {s} (m={m}, n={n}, q={q}, {'lds' if info['adm_in_lds'] else 'global'}): "
            f"ADM on the GPU's samples {rel:.2e}")
        assert rel <= 1e-3, f"slice {s}: {rel:.2e}"
    # (2) end to end
    w = run["r"]["WEIGHTS"]
    wo = {s: w[run["info"][s]["off_col"]: run["info"][s]["off_col"] + run["info"][s]["n"]].astype(np.uint64)
          for s in range(sc.n_slices)}
    I, per = orender.render(sc, p, weights_override=wo, keep=True)
    rows_all = np.concatenate([sc.slice_rows(s) for s in range(sc.n_slices)])
    rel_all = orender.relative_rmse(run["radiance"][rows_all], I[rows_all])
    log(f"batch frame: end-to-end pixel RMSE vs oracle {rel_all:.2e}")
    assert rel_all <= 1e-3
    noise = np.random.default_rng(5)
    for s in range(sc.n_slices):
        rows = sc.slice_rows(s)
        rel = orender.relative_rmse(run["radiance"][rows], I[rows])
        r = per[s]
        Ap = r["A"] * (1.0 + 1e-6 * noise.standard_normal(r["A"].shape))
        Ip, *_ = orender.complete_and_render(rows.shape[0], sc.slice_cols(s).shape[0], int(sc.rank[s]),
                                             r["ii"], r["jj"], Ap, 21, s, p)
        sens = orender.relative_rmse(Ip, r["I"])
        bound = min(CEILING, max(1e-3, 50.0 * sens))
        log(f"batch slice {s}: end-to-end {rel:.2e}, sensitivity to 1e-6 entry noise {sens:.2e}, bound {bound:.2e}")
        assert rel <= bound, f"slice {s} (m={rows.shape[0]}, q={sc.rank[s]}): {rel:.2e} > {bound:.2e}"
    outside = np.setdiff1d(np.arange(sc.m), sc.pt_ids)
    assert (run["radiance"][outside] == 0).all()


LOWQ = dataclasses.replace(CONFIGS["batch"], width=160, height=140, n_spheres=256, n_vpls=8000,
                           batch_slices=4, batch_m=(4700, 5200), batch_n=(256, 320), batch_q=(4, 8))


def test_low_rank_tall_slices_in_global_memory():
    """Ranks 4 and 8 on slices too tall for the LDS-resident kernel (m' q >
    18,432) complete in the global-memory kernel: the oracle's ADM on the
    GPU's samples against the GPU's radiance, 1e-3 pixel RMSE per slice."""
    sc = make_scene(LOWQ, 23)
    prm = api.default_params(seed=23, pass1_ppm=PPM, pass2_ppm=PPM, max_iter=40, fixed_iters=True)
    run = run_frame(sc, prm, label="tall low-rank slices")
    p = orender.Params(seed=23, pass1_ppm=PPM, pass2_ppm=PPM, max_iter=40, fixed_iters=True)
    ranks = set()
    for s in range(sc.n_slices):
        info = run["info"][s]
        m, n, q = info["m"], info["n"], info["q"]
        assert not info["adm_in_lds"], f"slice {s} (m={m}, q={q}) is not a global-memory slice"
        ranks.add(q)
        check_csr_csc(run, s)
        ii, jj, A = omega_of(run, s)
        I, *_ = orender.complete_and_render(m, n, q, ii, jj, A.astype(np.float64), 23, s, p)
        rel = orender.relative_rmse(run["radiance"][sc.slice_rows(s)], I)
        log(f"tall slice {s} (m={m}, n={n}, q={q}, global): ADM on the GPU's samples {rel:.2e}")
        assert rel <= 1e-3, f"slice {s}: {rel:.2e}"
    assert ranks == {4, 8}, ranks


@pytest.mark.parametrize("ppm", [5000, 50000])
def test_mid_other_rates(ppm):
    """The mid workload at 1% (0.5% + 0.5%) and 10% (5% + 5%): sampling
    properties of every slice, first and second pass bit-exact on two slices
    (the second given the GPU's weights), and the oracle's completion of the
    GPU's samples on the same two slices (100 fixed iterations, 1e-3)."""
    sc = make_scene("mid", SEED)
    prm = api.default_params(seed=SEED, pass1_ppm=ppm, pass2_ppm=ppm, fixed_iters=True)
    run = run_frame(sc, prm, label=f"mid {2 * ppm / 1e4:g}%")
    for s in range(sc.n_slices):
        info = run["info"][s]
        n = info["n"]
        i1, j1 = keys_to_ij(view(run, "OMEGA1", s))
        i2, j2 = keys_to_ij(view(run, "OMEGA2", s))
        assert np.unique(i1 * n + j1).shape[0] == info["N1"]
        assert np.unique(i2 * n + j2).shape[0] == info["N2"]
        assert not np.isin(i2 * n + j2, i1 * n + j1).any()
    p = orender.Params(seed=SEED, pass1_ppm=ppm, pass2_ppm=ppm, fixed_iters=True)
    for s in (3, 200):
        info = run["info"][s]
        m, n, q = info["m"], info["n"], info["q"]
        i1, j1 = pass1(SEED, s, m, n, ppm)
        gi, gj = keys_to_ij(view(run, "OMEGA1", s))
        assert np.array_equal(gi, i1) and np.array_equal(gj, j1)
        taken = np.zeros(m * n, bool)
        taken[gi * n + gj] = True
        w = view(run, "WEIGHTS", s).astype(np.uint64)
        i2, j2, short = pass2(SEED, s, m, n, info["N1"], ppm, w, taken)
        gi2, gj2 = keys_to_ij(view(run, "OMEGA2", s))
        assert np.array_equal(gi2, i2) and np.array_equal(gj2, j2) and not short
        ii, jj, A = omega_of(run, s)
        I, *_ = orender.complete_and_render(m, n, q, ii, jj, A.astype(np.float64), SEED, s, p)
        rel = orender.relative_rmse(run["radiance"][sc.slice_rows(s)], I)
        log(f"mid {2 * ppm / 1e4:g}% slice {s}: ADM on the GPU's samples {rel:.2e}")
        assert rel <= 1e-3
