"""Per-slice light coarsening (Sec. 4) on the GPU against the FP64 oracle, on
the tiny workload (1,024 singleton clusters under the light tree, 16 slices
of 256 rows, rank 8): the node table and the draw counts bit-exact, the merge
errors within FP32 shading tolerance, the merge decisions, columns and first
pass bit-exact given the GPU's merge errors, the second pass bit-exact given
the GPU's weights, and the coarsened frame within 1e-3 pixel RMSE of the
oracle's.  Also: no merge keeps the global cut, the bound mode's columns, and
a coarsened frame on the mid workload (4,096 clusters)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import check_scene_indices, entries_out_of_tol, keys_to_ij, log  # noqa: E402
from oracle import coarsen as C  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle.sampling import pass2  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene  # noqa: E402

SEED = 2
K = 4096          # row draws per slice (4 per leaf on average)
NMAX = 256        # columns per slice after coarsening
ITERS = 60
SLICES = (0, 5, 10, 15)

DT = {"LIGHTS": torch.float32, "REP": torch.int32, "BBOX": torch.float32, "NODE_MEMBERS": torch.int32,
      "LEAF_DRAWS": torch.int32, "NODE_EPS": torch.float32, "COLUMNS": torch.int32, "OMEGA1": torch.int32,
      "VAL1": torch.float32, "OMEGA2": torch.int32, "VAL2": torch.float32, "WEIGHTS": torch.int32}


def gpu_params(**kw):
    base = dict(seed=SEED, pass1_ppm=0, pass2_ppm=50000, max_iter=ITERS, fixed_iters=True)
    base.update(kw)
    return api.default_params(**base)


def oracle_params(**kw):
    base = dict(seed=SEED, pass1_ppm=0, pass2_ppm=50000, max_iter=ITERS, fixed_iters=True)
    base.update(kw)
    return orender.Params(**base)


def coarse_frame(sc, prm, co, label):
    check_scene_indices(sc)
    ng = sc.n_clusters
    assert sc.tree_left.shape == (ng - 1,) and sc.tree_right.shape == (ng - 1,)
    dev = torch.device("cuda", 0)
    log(f"coarsened frame {label}: m={sc.m} slices={sc.n_slices} leaves={ng} pixels={co.pixels} "
        f"n_max={co.n_max} bound={co.bound}")
    ctx = api.Context(0)
    ctx.set_occluders(sc.spheres)
    ds = api.DeviceScene(sc, dev)
    plan = api.Plan(sc, prm, co)
    ws = api.workspace(plan, dev)
    rad = api.render(ctx, plan, ds, prm, ws)
    torch.cuda.synchronize()
    out = dict(radiance=rad.double().cpu().numpy(), stats=api.read_stats(ctx, plan, ws),
               counts=api.read_counts(ctx, plan, ws), info=[plan.slice_info(s) for s in range(sc.n_slices)],
               r={k: api.region_view(plan, ws, k, dt).cpu().numpy() for k, dt in DT.items()},
               ctx=ctx, plan=plan, ws=ws, ds=ds)
    log(f"coarsened frame {label} done")
    return out


@pytest.fixture(scope="module")
def scene():
    return make_scene("tiny", SEED)


@pytest.fixture(scope="module")
def table(scene):
    return C.scene_table(scene, SEED)


@pytest.fixture(scope="module")
def run(scene):
    return coarse_frame(scene, gpu_params(), api.Coarsening(K, NMAX), "tiny")


def gpu_eps_of(run, s, ng):
    e = run["r"]["NODE_EPS"][s * (ng - 1): (s + 1) * (ng - 1)]
    full = np.zeros(2 * ng - 1, np.float32)
    full[ng:] = e
    return full


def test_node_table_and_draw_counts_bit_exact(scene, table, run):
    ng = scene.n_clusters
    NC = 2 * ng - 1
    L = run["r"]["LIGHTS"].reshape(9, NC)
    assert np.array_equal(run["r"]["REP"], table["rep"].astype(np.int32))
    V = scene.vpls
    for p, k in enumerate(("x", "y", "z", "nx", "ny", "nz")):
        assert np.array_equal(L[p], np.asarray(V[k], np.float32)[table["rep"]]), k
    assert np.array_equal(L[6:9].T, table["intensity"])
    B = run["r"]["BBOX"].reshape(6, NC)
    assert np.array_equal(B[:3].T, table["lo"]) and np.array_equal(B[3:].T, table["hi"])
    assert np.array_equal(run["r"]["NODE_MEMBERS"], table["members"].astype(np.int32))
    assert np.array_equal(run["r"]["LEAF_DRAWS"], C.leaf_quota(table["intensity"][:ng], K).astype(np.int32))
    log(f"node table: {NC} nodes bit-exact; draws per slice {int(run['r']['LEAF_DRAWS'].sum())}")


@pytest.mark.parametrize("s", SLICES)
def test_merge_errors_within_shading_tolerance(scene, table, run, s):
    ng = scene.n_clusters
    co = C.coarsen_slice(scene, table, s, SEED, C.CoarsenParams(pixels=K), NMAX, oracle_params())
    g = gpu_eps_of(run, s, ng)
    nodes = np.array(sorted(co["eps"]), np.int64)
    o = np.array([co["eps"][f] for f in nodes])
    amb = np.array([f in co["ambiguous_nodes"] for f in nodes])
    scale = max(float(o.max()), 1e-30)
    bad = (np.abs(g[nodes] - o) > 1e-4 * o + 1e-5 * scale) & ~amb
    log(f"slice {s}: {nodes.size} merge errors, max rel diff "
        f"{np.max(np.abs(g[nodes] - o) / np.maximum(o, 1e-5 * scale)):.2e}, {int(amb.sum())} ambiguous")
    assert not bad.any(), nodes[bad][:10]


@pytest.mark.parametrize("s", SLICES)
def test_columns_and_first_pass_bit_exact_given_gpu_errors(scene, table, run, s):
    ng = scene.n_clusters
    co = C.coarsen_slice(scene, table, s, SEED, C.CoarsenParams(pixels=K), NMAX, oracle_params(),
                         eps_override=gpu_eps_of(run, s, ng))
    info = run["info"][s]
    n, N1 = int(run["counts"]["n"][s]), int(run["counts"]["N1"][s])
    assert n == co["n"] == min(ng, max(NMAX, int(scene.rank[s])))
    cols = run["r"]["COLUMNS"][info["off_col"]: info["off_col"] + n]
    assert np.array_equal(cols, co["columns"])
    i1, j1 = keys_to_ij(run["r"]["OMEGA1"][info["off1"]: info["off1"] + N1])
    assert N1 == co["i1"].shape[0] <= info["N1"]
    assert np.array_equal(i1, co["i1"]) and np.array_equal(j1, co["j1"])
    # entries of the coarsened first pass (node lights)
    L = C.node_lights(scene, table)
    A1, amb, _ = orender.eval_entries(scene, L, scene.slice_rows(s)[i1], co["columns"][j1], oracle_params())
    v1 = run["r"]["VAL1"][3 * info["off1"]: 3 * (info["off1"] + N1)].reshape(-1, 3)
    assert not entries_out_of_tol(v1, A1, amb).any()
    log(f"slice {s}: {n} columns, {N1} first-pass entries bit-exact")


@pytest.mark.parametrize("s", SLICES)
def test_second_pass_and_radiance_given_gpu_errors_and_weights(scene, table, run, s):
    ng = scene.n_clusters
    info = run["info"][s]
    n, N1 = int(run["counts"]["n"][s]), int(run["counts"]["N1"][s])
    m = info["m"]
    w = run["r"]["WEIGHTS"][info["off_col"]: info["off_col"] + n].astype(np.uint64)
    i1, j1 = keys_to_ij(run["r"]["OMEGA1"][info["off1"]: info["off1"] + N1])
    taken = np.zeros(m * n, bool)
    taken[i1 * n + j1] = True
    i2, j2, short = pass2(SEED, s, m, n, N1, 50000, w, taken)
    n2 = int(run["stats"]["n2"][s])
    assert n2 == i2.shape[0] == int(run["counts"]["N2"][s]) and not short
    g2i, g2j = keys_to_ij(run["r"]["OMEGA2"][info["off2"]: info["off2"] + n2])
    assert np.array_equal(g2i, i2) and np.array_equal(g2j, j2)
    r = C.render_slice_coarsened(scene, table, s, oracle_params(), C.CoarsenParams(pixels=K), NMAX,
                                 weights_override=w, eps_override=gpu_eps_of(run, s, ng))
    rows = scene.slice_rows(s)
    rel = orender.relative_rmse(run["radiance"][rows], r["I"])
    log(f"slice {s}: second pass {n2} bit-exact; pixel RMSE vs oracle {rel:.2e}")
    assert rel <= 1e-3


def test_no_merge_keeps_the_global_cut(scene, table):
    ng = scene.n_clusters
    run = coarse_frame(scene, gpu_params(max_iter=5), api.Coarsening(2048, ng), "tiny, no merge")
    for s in (0, 7):
        info = run["info"][s]
        assert int(run["counts"]["n"][s]) == ng
        assert np.array_equal(run["r"]["COLUMNS"][info["off_col"]: info["off_col"] + ng], np.arange(ng))
        co = C.coarsen_slice(scene, table, s, SEED, C.CoarsenParams(pixels=2048), ng, oracle_params(),
                             eps_override=gpu_eps_of(run, s, ng))
        N1 = int(run["counts"]["N1"][s])
        i1, j1 = keys_to_ij(run["r"]["OMEGA1"][info["off1"]: info["off1"] + N1])
        assert np.array_equal(i1, co["i1"]) and np.array_equal(j1, co["j1"])


def test_bound_mode_columns(scene, table, run):
    """Merging while the cost stays below a bound (no target count): the
    column count is the frame's own; columns bit-exact given the GPU's errors."""
    ng = scene.n_clusters
    eps0 = run["r"]["NODE_EPS"][: ng - 1]
    bound = float(np.quantile(eps0[eps0 > 0], 0.3))
    run_b = coarse_frame(scene, gpu_params(max_iter=5), api.Coarsening(K, ng, bound), "tiny, bound")
    ns = []
    for s in SLICES:
        info = run_b["info"][s]
        n = int(run_b["counts"]["n"][s])
        co = C.coarsen_slice(scene, table, s, SEED, C.CoarsenParams(pixels=K, bound=bound), ng, oracle_params(),
                             eps_override=gpu_eps_of(run_b, s, ng))
        assert n == co["n"]
        assert np.array_equal(run_b["r"]["COLUMNS"][info["off_col"]: info["off_col"] + n], co["columns"])
        ns.append(n)
    log(f"bound {bound:.3e}: columns per slice {ns}")
    assert min(ns) < ng


def test_mid_frame_coarsened(tmp_path):
    """Mid workload (512 x 512, 4,096-cluster cut, rank 16) coarsened to at most
    512 columns per slice: every slice's counts, and one slice's columns and
    first pass bit-exact given the GPU's errors."""
    sc = make_scene("mid", 11)
    prm = gpu_params(seed=11, pass2_ppm=25000, max_iter=20)
    co_spec = api.Coarsening(16384, 512)
    run = coarse_frame(sc, prm, co_spec, "mid")
    ng = sc.n_clusters
    n = run["counts"]["n"]
    assert np.all(n == np.minimum(ng, np.maximum(512, sc.rank)))
    assert np.all(run["counts"]["N1"] > 0) and np.all(run["counts"]["N1"] <= 16384)
    assert np.all(run["stats"]["n2"] == run["counts"]["N2"])
    assert np.all(np.isfinite(run["radiance"]))
    table = C.scene_table(sc, 11)
    s = 37
    co = C.coarsen_slice(sc, table, s, 11, C.CoarsenParams(pixels=16384), 512,
                         orender.Params(seed=11), eps_override=gpu_eps_of(run, s, ng))
    info = run["info"][s]
    assert np.array_equal(run["r"]["COLUMNS"][info["off_col"]: info["off_col"] + int(n[s])], co["columns"])
    N1 = int(run["counts"]["N1"][s])
    i1, j1 = keys_to_ij(run["r"]["OMEGA1"][info["off1"]: info["off1"] + N1])
    assert np.array_equal(i1, co["i1"]) and np.array_equal(j1, co["j1"])
    log(f"mid: {sc.n_slices} slices coarsened to {int(n.min())}..{int(n.max())} columns, "
        f"first pass {int(run['counts']['N1'].sum())} entries")


def test_frame_totals_count_every_evaluation(scene, table, run):
    """vplmc_read_totals: the sampled entries of both passes, and exactly one
    coarsening evaluation per drawn row and level, from its leaf to the root
    (min(m', k_x) draws of leaf x, each walking depth(x) + 1 nodes)."""
    ng = scene.n_clusters
    tot = api.read_totals(run["ctx"], run["plan"], run["ws"])
    assert tot["entries"] == int(run["counts"]["N1"].sum() + run["stats"]["n2"].sum())
    depth = np.zeros(ng, np.int64)
    for x in range(ng):
        y = x
        while table["parent"][y] >= 0:
            y = table["parent"][y]
            depth[x] += 1
    k = run["r"]["LEAF_DRAWS"].astype(np.int64)
    want = sum(int((np.minimum(k, info["m"]) * (depth + 1)).sum()) for info in run["info"])
    assert tot["coarsen_evals"] == want
    assert 0 < tot["coarsen_rays"] <= tot["coarsen_evals"] and 0 < tot["rays"] <= tot["entries"]
    log(f"totals: {tot}")
