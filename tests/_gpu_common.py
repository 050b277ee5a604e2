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


def within_entry_tol(g, o, amb=None):
    """|g - o| <= 1e-4 |o| + 1e-7 max|o| per entry and channel (unflagged entries)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    tol = 1e-4 * np.abs(o) + 1e-7 * max(np.abs(o).max(), 1e-30)
    bad = np.abs(g - o) > tol
    if amb is not None:
        bad &= ~np.asarray(amb, bool)[:, None]
    return bad
