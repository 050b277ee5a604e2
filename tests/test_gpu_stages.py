"""The stage calls of the C ABI on the GPU against the FP64 oracle: every
entry of two tiny slices (vplmc_full_matrix); the second pass given weights,
including maximal and arbitrary 32-bit weights on slices of 1,024 columns
(vplmc_stage_pass2); the completion from caller samples and caller initial
factors at fixed iterations against the oracle's ADM from the same start, and
planted low-rank recovery (vplmc_stage_adm, Appendix A); the factorised sum
(vplmc_stage_reduce); malformed samples rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import entries_out_of_tol, keys_to_ij, log  # noqa: E402
from oracle import adm as oadm  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle.sampling import count_from_ppm, pass2  # noqa: E402
from paper_2202_12567_amd import _native as N  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene  # noqa: E402

SEED = 5
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def scene():
    return make_scene("tiny", SEED)


@pytest.fixture(scope="module")
def frame(scene):
    """One plain tiny frame (its OMEGA1, X, Y, SLICE_SCALE stay in the workspace)."""
    prm = api.default_params(seed=SEED, max_iter=30, fixed_iters=True)
    ctx = api.Context(0)
    ctx.set_occluders(scene.spheres)
    ds = api.DeviceScene(scene, DEV)
    plan = api.Plan(scene, prm)
    ws = api.workspace(plan, DEV)
    log("stage tests: tiny frame")
    rad = api.render(ctx, plan, ds, prm, ws).clone()
    torch.cuda.synchronize()
    return dict(ctx=ctx, ds=ds, plan=plan, ws=ws, prm=prm, rad=rad)


def test_full_matrix_matches_oracle(scene, frame):
    lights = api.region_view(frame["plan"], frame["ws"], "LIGHTS", torch.float32).view(9, -1)
    A = api.full_matrix(frame["ctx"], frame["plan"], frame["ds"], lights, frame["prm"], 3, 5).cpu().numpy()
    L = orender.cluster_lights(scene, SEED)
    got, want, amb = [], [], []
    o = 0
    for s in (3, 4):
        rows, cols = scene.slice_rows(s), scene.slice_cols(s)
        ii, jj = np.meshgrid(np.arange(rows.shape[0]), np.arange(cols.shape[0]), indexing="ij")
        a, b, _ = orender.eval_entries(scene, L, rows[ii.ravel()], cols[jj.ravel()], orender.Params(seed=SEED))
        k = rows.shape[0] * cols.shape[0]
        got.append(A[o: o + k])
        want.append(a)
        amb.append(b)
        o += k
    assert o == A.shape[0]
    bad = entries_out_of_tol(np.concatenate(got), np.concatenate(want), np.concatenate(amb))
    log(f"full matrix: {o} entries, {int(np.concatenate(amb).sum())} ambiguous, {int(bad.sum())} out of tolerance")
    assert not bad.any()


def test_stage_pass2_given_weights_bit_exact(scene, frame):
    """Weights of 2^24 on every column (a 256-column chunk sums to 2^32), arbitrary
    32-bit weights, zeros with a few non-zero columns: the second pass equals
    the oracle's, attempt for attempt."""
    plan, ws, ctx = frame["plan"], frame["ws"], frame["ctx"]
    rng = np.random.default_rng(3)
    wv = api.region_view(plan, ws, "WEIGHTS", torch.int32)
    cases = {}
    for s in range(scene.n_slices):
        info = plan.slice_info(s)
        n = info["n"]
        if s % 3 == 0:
            w = np.full(n, 1 << 24, np.uint64)
        elif s % 3 == 1:
            w = rng.integers(0, 1 << 32, n, dtype=np.uint64)
        else:
            w = np.zeros(n, np.uint64)
            w[rng.choice(n, 5, replace=False)] = rng.integers(1, 1 << 20, 5, dtype=np.uint64)
        cases[s] = w
        wv[info["off_col"]: info["off_col"] + n] = torch.as_tensor(w.astype(np.uint32).view(np.int32), device=DEV)
    api.stage_pass2(ctx, plan, frame["prm"], ws)
    st = api.read_stats(ctx, plan, ws)
    om1 = api.region_view(plan, ws, "OMEGA1", torch.int32).cpu().numpy()
    om2 = api.region_view(plan, ws, "OMEGA2", torch.int32).cpu().numpy()
    for s, w in cases.items():
        info = plan.slice_info(s)
        m, n = info["m"], info["n"]
        i1, j1 = keys_to_ij(om1[info["off1"]: info["off1"] + info["N1"]])
        taken = np.zeros(m * n, bool)
        taken[i1 * n + j1] = True
        i2, j2, short = pass2(SEED, s, m, n, info["N1"], frame["prm"].pass2_ppm, w, taken)
        n2 = int(st["n2"][s])
        gi, gj = keys_to_ij(om2[info["off2"]: info["off2"] + n2])
        assert n2 == i2.shape[0], s
        assert np.array_equal(gi, i2) and np.array_equal(gj, j2), s
        assert bool(st["flags"][s] & N.SLICE_SHORTFALL) == bool(short), s
    log(f"stage pass 2: {len(cases)} slices bit-exact (maximal, 32-bit and sparse weights)")


def planted(m, n, r, seed):
    rng = np.random.default_rng(seed)
    Xs = rng.uniform(0, 1, (m, r))
    Ys = rng.uniform(0, 1, (r, 3 * n))
    return Xs @ Ys


def stage_plan(m, n, q, ppm, ctx):
    class One:
        n_slices, n_clusters = 1, n
        pt_offsets = np.array([0, m], np.int32)
        cl_offsets = np.array([0, n], np.int32)
        rank = np.array([q], np.int32)
    prm = api.default_params(seed=SEED, pass1_ppm=ppm, pass2_ppm=0)
    plan = api.Plan(One, prm)
    return plan, api.workspace(plan, DEV)


def put_samples(plan, ws, M, n, ii, jj):
    keys = (ii.astype(np.int64) << 16) | jj.astype(np.int64)
    api.region_view(plan, ws, "OMEGA1", torch.int32)[: ii.shape[0]] = torch.as_tensor(
        keys.astype(np.uint32).view(np.int32), device=DEV)
    vals = np.stack([M[ii, jj + c * n] for c in range(3)], axis=1).astype(np.float32)
    api.region_view(plan, ws, "VAL1", torch.float32)[: 3 * ii.shape[0]] = torch.as_tensor(vals.ravel(), device=DEV)
    return vals


def factors_of(plan, ws, m, n, q):
    info = plan.slice_info(0)
    qp = info["q_pad"]
    X = api.region_view(plan, ws, "X", torch.float32)[: m * qp].cpu().numpy().reshape(m, qp).astype(np.float64)
    Yg = api.region_view(plan, ws, "Y", torch.float32)[: 3 * n * qp].cpu().numpy().reshape(n, 3, qp)
    Y = np.transpose(Yg, (2, 1, 0)).reshape(qp, 3 * n).astype(np.float64)      # Y[k, c n + j]
    s0 = float(api.region_view(plan, ws, "SLICE_SCALE", torch.float32)[0].item())
    assert not X[:, q:].any() and not Y[q:].any()
    return X[:, :q], Y[:q], s0


def test_stage_adm_from_given_factors_matches_oracle(frame):
    """Caller samples (40% of a 48 x 40 slice, all three channels) and caller
    initial factors: 300 fixed iterations on the GPU against the oracle's ADM
    from the same FP32 start, over every entry of the stacked matrix."""
    m, n, q = 48, 40, 3
    ctx = frame["ctx"]
    ppm = 400000
    plan, ws = stage_plan(m, n, q, ppm, ctx)
    N1 = plan.slice_info(0)["N1"]
    assert N1 == count_from_ppm(ppm, m * n)
    M = planted(m, n, q, 11)
    rng = np.random.default_rng(12)
    e = np.sort(rng.choice(m * n, N1, replace=False))
    ii, jj = e // n, e % n
    vals = put_samples(plan, ws, M, n, ii, jj)
    rs = np.random.default_rng(13)
    X0 = rs.uniform(0, 1, (m, q)).astype(np.float32)
    Y0 = rs.uniform(0, 1, (q, 3 * n)).astype(np.float32)
    qp = plan.slice_info(0)["q_pad"]
    Xg = np.zeros((m, qp), np.float32)
    Xg[:, :q] = X0
    Yg = np.zeros((n, 3, qp), np.float32)
    Yg[:, :, :q] = np.transpose(Y0.reshape(q, 3, n), (2, 1, 0))
    api.region_view(plan, ws, "X", torch.float32)[: m * qp] = torch.as_tensor(Xg.ravel(), device=DEV)
    api.region_view(plan, ws, "Y", torch.float32)[: 3 * n * qp] = torch.as_tensor(Yg.ravel(), device=DEV)
    prm = api.default_params(seed=SEED, pass1_ppm=ppm, pass2_ppm=0, max_iter=300, fixed_iters=True, given_init=True)
    pt = torch.arange(m, dtype=torch.int32, device=DEV)
    rad = api.stage_adm(ctx, plan, prm, pt, ws, n_points=m).double().cpu().numpy()
    X, Y, s0 = factors_of(plan, ws, m, n, q)
    I, iters, err, flags, fac = orender.complete_and_render(
        m, n, q, ii, jj, vals.astype(np.float64), SEED, 0,
        orender.Params(seed=SEED, max_iter=300, fixed_iters=True), X0Y0=(X0.astype(np.float64), Y0.astype(np.float64)))
    Xo, Yo, s0o = fac
    assert abs(s0 - s0o) <= 1e-6 * s0o
    full_g = s0 * X @ Y
    full_o = s0o * Xo @ Yo
    rel = np.linalg.norm(full_g - full_o) / np.linalg.norm(full_o)
    rel_I = orender.relative_rmse(rad, I)
    log(f"stage ADM from given factors, 300 iterations: stacked matrix vs oracle {rel:.2e}, radiance {rel_I:.2e}")
    assert rel <= 1e-3 and rel_I <= 1e-3


def test_stage_adm_recovers_a_planted_low_rank_matrix(frame):
    """Planted rank-3 stacked matrix, 40% of the entries observed, rank 3 (run
    at the kernels' rank 4 with one zero component), up to 3,000 iterations
    with tol 1e-7: the whole matrix, unobserved entries included, is recovered
    to FP32 accuracy."""
    m, n, q = 48, 40, 3
    ctx = frame["ctx"]
    ppm = 400000
    plan, ws = stage_plan(m, n, q, ppm, ctx)
    N1 = plan.slice_info(0)["N1"]
    M = planted(m, n, q, 21)
    rng = np.random.default_rng(22)
    e = np.sort(rng.choice(m * n, N1, replace=False))
    put_samples(plan, ws, M, n, e // n, e % n)
    prm = api.default_params(seed=SEED, pass1_ppm=ppm, pass2_ppm=0, max_iter=3000, tol=1e-7)
    pt = torch.arange(m, dtype=torch.int32, device=DEV)
    api.stage_adm(ctx, plan, prm, pt, ws, n_points=m)
    X, Y, s0 = factors_of(plan, ws, m, n, q)
    st = api.read_stats(ctx, plan, ws)
    rel = np.linalg.norm(s0 * X @ Y - M) / np.linalg.norm(M)
    log(f"planted rank 3: {int(st['iters'][0])} iterations, residual {float(st['resid'][0]):.2e}, "
        f"whole-matrix error {rel:.2e}")
    assert rel < 1e-4


def test_stage_reduce_reproduces_the_frame(scene, frame):
    plan, ws, ctx = frame["plan"], frame["ws"], frame["ctx"]
    # (the pass-2 test above changed OMEGA2 but not X, Y or the scale)
    rad = api.stage_reduce(ctx, plan, frame["ds"].pt_ids, scene.m, ws)
    assert torch.equal(rad, frame["rad"])
    info = plan.slice_info(2)
    qp, m, n = info["q_pad"], info["m"], info["n"]
    X = api.region_view(plan, ws, "X", torch.float32)[info["off_x"]: info["off_x"] + m * qp].cpu().numpy()
    Y = api.region_view(plan, ws, "Y", torch.float32)[info["off_y"]: info["off_y"] + 3 * n * qp].cpu().numpy()
    s0 = float(api.region_view(plan, ws, "SLICE_SCALE", torch.float32)[2].item())
    w = Y.reshape(n, 3, qp).astype(np.float64).sum(axis=0)          # (3, qp)
    want = s0 * X.reshape(m, qp).astype(np.float64) @ w.T
    got = rad.double().cpu().numpy()[scene.slice_rows(2)]
    assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()


def test_stage_rejects_malformed_samples(frame):
    m, n, q = 48, 40, 3
    ctx = frame["ctx"]
    plan, ws = stage_plan(m, n, q, 400000, ctx)
    N1 = plan.slice_info(0)["N1"]
    prm = api.default_params(seed=SEED, pass1_ppm=400000, pass2_ppm=0, max_iter=5)
    pt = torch.arange(m, dtype=torch.int32, device=DEV)
    om = api.region_view(plan, ws, "OMEGA1", torch.int32)
    base = np.arange(N1, dtype=np.int64)
    keys = ((base // n) << 16) | (base % n)
    keys[7] = keys[3]                                  # a repeated entry
    om[:N1] = torch.as_tensor(keys.astype(np.uint32).view(np.int32), device=DEV)
    with pytest.raises(N.VplmcError) as e:
        api.stage_adm(ctx, plan, prm, pt, ws, n_points=m)
    assert e.value.code == N.EINVAL
    keys = ((base // n) << 16) | (base % n)
    keys[0] = (m << 16) | 0                            # a row outside the slice
    om[:N1] = torch.as_tensor(keys.astype(np.uint32).view(np.int32), device=DEV)
    with pytest.raises(N.VplmcError) as e:
        api.stage_adm(ctx, plan, prm, pt, ws, n_points=m)
    assert e.value.code == N.EINVAL
