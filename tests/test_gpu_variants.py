"""Completion variants on the GPU against the FP64 oracle (tiny workload,
16 slices of 256 rows and 1,024 columns): per-row masked ALS (VPLMC_ALS) at
its own rank and at ranks padded to the kernels' (3, 5, 12, 20), and the ADM
with its non-negativity switched off (VPLMC_NO_NONNEG); each from the GPU's
own samples through the oracle's completion, pixel RMSE <= 1e-3 per slice."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import log, omega_of, run_frame  # noqa: E402
from oracle import render as orender  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene, scene_sample  # noqa: E402

SEED = 3
ITERS = 40


@pytest.fixture(scope="module")
def scene():
    return make_scene("tiny", SEED)


def check_against_oracle(sc, r, label, **oracle_kw):
    worst = 0.0
    for s in range(sc.n_slices):
        info = r["info"][s]
        ii, jj, A = omega_of(r, s)
        I, iters, err, flags, fac = orender.complete_and_render(
            info["m"], info["n"], info["q"], ii, jj, A.astype(np.float64), SEED, s,
            orender.Params(seed=SEED, max_iter=ITERS, fixed_iters=True, **oracle_kw))
        rel = orender.relative_rmse(r["radiance"][sc.slice_rows(s)], I)
        worst = max(worst, rel)
        assert rel <= 1e-3, f"{label}, slice {s}: pixel RMSE {rel:.2e}"
        assert abs(float(r["stats"]["resid"][s]) - err) <= 1e-3 * err + 1e-6, (label, s)
    log(f"{label}: worst slice pixel RMSE vs oracle {worst:.2e}")


def test_masked_als_matches_oracle(scene):
    prm = api.default_params(seed=SEED, max_iter=ITERS, fixed_iters=True, als=True)
    r = run_frame(scene, prm, label="masked ALS")
    assert all(not i["adm_in_lds"] for i in r["info"])
    check_against_oracle(scene, r, "masked ALS, rank 8", method="als", lam=0.01)


def test_masked_als_at_padded_ranks(scene):
    ranks = [3, 5, 12, 20]
    sub = scene_sample(scene, list(range(len(ranks))))
    sub.rank = np.asarray(ranks, np.int32)
    prm = api.default_params(seed=SEED, max_iter=ITERS, fixed_iters=True, als=True)
    r = run_frame(sub, prm, label="masked ALS ranks 3-20")
    check_against_oracle(sub, r, "masked ALS, ranks 3/5/12/20", method="als", lam=0.01)


def test_adm_without_nonnegativity_matches_oracle(scene):
    prm = api.default_params(seed=SEED, max_iter=ITERS, fixed_iters=True, no_nonneg=True)
    r = run_frame(scene, prm, label="ADM, non-negativity off")
    check_against_oracle(scene, r, "ADM without non-negativity", nonneg=False)


def test_variants_differ_and_converge_in_tolerance_mode(scene):
    """Tolerance mode (no fixed count): every variant reports iterations and a
    residual; the plan and the frame must agree on the method."""
    out = {}
    for name, kw in (("adm", {}), ("no_nonneg", dict(no_nonneg=True)), ("als", dict(als=True))):
        prm = api.default_params(seed=SEED, max_iter=100, tol=1e-3, **kw)
        r = run_frame(scene, prm, regions=False, label=f"{name} tol")
        out[name] = r["radiance"]
        assert np.all(r["stats"]["iters"] <= 100) and np.all(np.isfinite(r["stats"]["resid"]))
    assert not np.array_equal(out["adm"], out["als"]) and not np.array_equal(out["adm"], out["no_nonneg"])
    # a frame whose method differs from its plan's is refused
    plan = api.Plan(scene, api.default_params(seed=SEED))
    ws = api.workspace(plan, torch.device("cuda", 0))
    ctx = api.Context(0)
    ds = api.DeviceScene(scene, torch.device("cuda", 0))
    with pytest.raises(api.N.VplmcError):
        api.render(ctx, plan, ds, api.default_params(seed=SEED, als=True), ws)
