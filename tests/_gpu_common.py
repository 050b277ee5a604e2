"""Shared helpers of the GPU parity tests: run the HIP path once on a scene
and pull every intermediate region back to the host."""
import sys

import numpy as np
import torch

from paper_2202_12567_amd import api
from scenegen import make_scene

REGION_DTYPES = {
    "LIGHTS": torch.float32, "REP": torch.int32, "BBOX": torch.float32, "OMEGA1": torch.int32,
    "VAL1": torch.float32, "OMEGA2": torch.int32, "VAL2": torch.float32, "WEIGHTS": torch.int32,
    "COLMIN": torch.float32, "COLMAX": torch.float32, "COLCNT": torch.int32, "ROW_PTR": torch.int32,
    "CSR_COL": torch.int32, "CSR_VAL": torch.float32, "COL_PTR": torch.int32, "CSC_ROW": torch.int32,
    "CSC_VAL": torch.float32, "X": torch.float32, "Y": torch.float32, "SLICE_SCALE": torch.float32,
    "FEATURES": torch.float32, "LOGITS": torch.float32,
}


def log(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def check_scene_indices(sc):
    """Host-side bounds check of every index the kernels will follow."""
    assert sc.pt_ids.min() >= 0 and sc.pt_ids.max() < sc.m
    assert sc.cl_ids.min() >= 0 and sc.cl_ids.max() < sc.n_clusters
    assert sc.cut_members.min() >= 0 and sc.cut_members.max() < sc.n
    assert sc.cut_offsets[0] == 0 and sc.cut_offsets[-1] == sc.cut_members.shape[0]
    assert np.all(np.diff(sc.cut_offsets) >= 1)
    assert sc.pt_offsets[-1] == sc.pt_ids.shape[0] and sc.cl_offsets[-1] == sc.cl_ids.shape[0]


def run_frame(sc, params, regions=True, label=""):
    check_scene_indices(sc)
    dev = torch.device("cuda", 0)
    log(f"render {label} m={sc.m} slices={sc.n_slices} clusters={sc.n_clusters} "
        f"ppm={params.pass1_ppm}+{params.pass2_ppm} max_iter={params.max_iter}")
    ctx = api.Context(0)
    ctx.set_occluders(sc.spheres)
    ds = api.DeviceScene(sc, dev)
    plan = api.Plan(sc, params)
    ws = api.workspace(plan, dev)
    rad = api.render(ctx, plan, ds, params, ws)
    torch.cuda.synchronize()
    out = dict(radiance=rad.double().cpu().numpy(), stats=api.read_stats(ctx, plan, ws),
               info=[plan.slice_info(s) for s in range(sc.n_slices)], ctx=ctx, ds=ds, plan=plan, ws=ws)
    if regions:
        out["r"] = {k: api.region_view(plan, ws, k, dt).cpu().numpy() for k, dt in REGION_DTYPES.items()}
    log(f"render {label} done")
    return out


def keys_to_ij(keys):
    keys = np.asarray(keys).astype(np.int64) & 0xFFFFFFFF
    return keys >> 16, keys & 0xFFFF


def omega_of(run, s):
    """Rows, columns and FP32 RGB values of slice s's samples (both passes, draw
    and acceptance order), from the passes' own output regions."""
    info = run["info"][s]
    n2 = int(run["stats"]["n2"][s])
    k1 = run["r"]["OMEGA1"][info["off1"]: info["off1"] + info["N1"]]
    k2 = run["r"]["OMEGA2"][info["off2"]: info["off2"] + n2]
    v1 = run["r"]["VAL1"][3 * info["off1"]: 3 * (info["off1"] + info["N1"])]
    v2 = run["r"]["VAL2"][3 * info["off2"]: 3 * (info["off2"] + n2)]
    i, j = keys_to_ij(np.concatenate([k1, k2]))
    return i, j, np.concatenate([v1, v2]).reshape(-1, 3)


def check_csr_csc(run, s):
    """CSR and CSC copies of a slice completed in global memory: row-major and
    column-major orders of exactly the passes' samples."""
    info = run["info"][s]
    m, n = info["m"], info["n"]
    i, j, v = omega_of(run, s)
    nnz = i.shape[0]
    o = info["off_omega"]
    order = np.lexsort((j, i))
    rp = np.concatenate([[0], np.cumsum(np.bincount(i, minlength=m))])
    assert np.array_equal(run["r"]["ROW_PTR"][info["off_row"]: info["off_row"] + m + 1], rp)
    assert np.array_equal(run["r"]["CSR_COL"][o: o + nnz], j[order])
    assert np.array_equal(run["r"]["CSR_VAL"][3 * o: 3 * (o + nnz)].reshape(-1, 3), v[order])
    order = np.lexsort((i, j))
    cp = np.concatenate([[0], np.cumsum(np.bincount(j, minlength=n))])
    assert np.array_equal(run["r"]["COL_PTR"][info["off_colptr"]: info["off_colptr"] + n + 1], cp)
    assert np.array_equal(run["r"]["CSC_ROW"][o: o + nnz], i[order])
    assert np.array_equal(run["r"]["CSC_VAL"][3 * o: 3 * (o + nnz)].reshape(-1, 3), v[order])


def entries_out_of_tol(g, o, amb=None):
    """|g - o| <= 1e-4 |o| + 1e-7 max|o| per entry and channel (unflagged entries)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    tol = 1e-4 * np.abs(o) + 1e-7 * max(np.abs(o).max(), 1e-30)
    bad = np.abs(g - o) > tol
    if amb is not None:
        bad &= ~np.asarray(amb, bool)[:, None]
    return bad
