"""Python binding of libvplmc (include/vplmc.h).

Argument marshalling only: PyTorch provides device memory and the stream,
and every step of the method runs in the library's HIP kernels.  The
function names follow the C entry points without the ``vplmc_`` prefix.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N
from ._native import check


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else int(t.data_ptr()))


def version():
    return N.load().vplmc_version()


def default_params(fixed_iters=None, learned=None, features=None, given_init=None, no_nonneg=None, als=None, **kw):
    """vplmc_default_params with overrides; booleans toggle the flag bits."""
    p = N.Params()
    check(N.load().vplmc_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    for bit, on in ((N.FIXED_ITERS, fixed_iters), (N.LEARNED, learned), (N.FEATURES, features),
                    (N.GIVEN_INIT, given_init), (N.NO_NONNEG, no_nonneg), (N.ALS, als)):
        if on is not None:
            p.flags = (p.flags | bit) if on else (p.flags & ~bit)
    return p


def bvh_build(spheres):
    """vplmc_bvh_build: (boxes (n_nodes, 6), codes (n_nodes, 2), sphere order (n,)) of the sphere BVH; host only."""
    lib = N.load()
    cx, cy, cz, r = (np.ascontiguousarray(spheres[k], dtype=np.float32) for k in ("cx", "cy", "cz", "r"))
    f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    n = int(cx.shape[0])
    nn = ctypes.c_int32()
    lib.vplmc_bvh_build(n, f(cx), f(cy), f(cz), f(r), 0, None, None, None, ctypes.byref(nn))
    box = np.zeros((max(nn.value, 1), 6), np.float32)
    code = np.zeros((max(nn.value, 1), 2), np.int32)
    order = np.zeros(max(n, 1), np.int32)
    check(lib.vplmc_bvh_build(n, f(cx), f(cy), f(cz), f(r), nn.value, f(box), f(code), f(order), ctypes.byref(nn)))
    return box[:nn.value], code[:nn.value], order[:n]


def sbvh_build(tri):
    """vplmc_sbvh_build: (boxes (n_nodes, 6), codes (n_nodes, 2), refs (n_refs,)) of the SBVH over
    triangles (T, 9); host only."""
    lib = N.load()
    tri = np.ascontiguousarray(tri, dtype=np.float32).reshape(-1, 9)
    f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    nn, nr = ctypes.c_int32(), ctypes.c_int32()
    lib.vplmc_sbvh_build(int(tri.shape[0]), f(tri), 0, None, None, 0, None, ctypes.byref(nn), ctypes.byref(nr))
    box = np.zeros((max(nn.value, 1), 6), np.float32)
    code = np.zeros((max(nn.value, 1), 2), np.int32)
    refs = np.zeros(max(nr.value, 1), np.int32)
    check(lib.vplmc_sbvh_build(int(tri.shape[0]), f(tri), nn.value, f(box), f(code), nr.value, f(refs),
                               ctypes.byref(nn), ctypes.byref(nr)))
    return box[:nn.value], code[:nn.value], refs[:nr.value]


class Context:
    """Device + stream (vplmc_create).  The stream defaults to torch's current stream."""

    def __init__(self, device=0, stream=None):
        lib = N.load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib.vplmc_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def set_occluders(self, spheres):
        """Spheres (cx, cy, cz, r), or triangles under the key "tri" ((T, 9) v0 v1 v2)."""
        f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        if "tri" in spheres:
            tri = np.ascontiguousarray(spheres["tri"], dtype=np.float32).reshape(-1, 9)
            check(N.load().vplmc_set_triangles(self.h, int(tri.shape[0]), f(tri)))
            return
        cx, cy, cz, r = (np.ascontiguousarray(spheres[k], dtype=np.float32) for k in ("cx", "cy", "cz", "r"))
        check(N.load().vplmc_set_occluders(self.h, int(cx.shape[0]), f(cx), f(cy), f(cz), f(r)))

    def close(self):
        if self.h:
            N.load().vplmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceScene:
    """Device copies of a scene's arrays plus the C structs that point at them."""

    POINT_KEYS = ("px", "py", "pz", "nx", "ny", "nz", "kd_r", "kd_g", "kd_b", "ks", "phong_e")
    LIGHT_KEYS = ("x", "y", "z", "nx", "ny", "nz", "ir", "ig", "ib")

    def __init__(self, scene, device):
        dev = torch.device(device)
        t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
        self.scene = scene
        self.pts = {k: t(scene.points[k]) for k in self.POINT_KEYS}
        self.vpl = {k: t(scene.vpls[k]) for k in self.LIGHT_KEYS}
        self.cut_offsets = t(scene.cut_offsets, torch.int32)
        self.cut_members = t(scene.cut_members, torch.int32)
        self.pt_ids = t(scene.pt_ids, torch.int32)
        self.cl_ids = t(scene.cl_ids, torch.int32)
        self.m = scene.m
        self.n_vpls = scene.n
        self.n_clusters = scene.n_clusters
        self.points_c = N.Points(self.m, *[_ptr(self.pts[k]) for k in self.POINT_KEYS], None, None, None)
        self.vpls_c = lights_struct(self.vpl)
        self.cut_c = N.Cut(self.n_clusters, _ptr(self.cut_offsets), _ptr(self.cut_members))


def lights_struct(d):
    """C struct for a dict of 9 light planes (x y z nx ny nz ir ig ib) or a (9, n) tensor."""
    if isinstance(d, torch.Tensor):
        d = {k: d[i] for i, k in enumerate(DeviceScene.LIGHT_KEYS)}
    n = int(d["x"].shape[0])
    return N.Lights(n, *[_ptr(d[k]) for k in DeviceScene.LIGHT_KEYS])


class Coarsening:
    """Light coarsening of every slice (Sec. 4): `pixels` row draws per slice,
    column cap n_max (int or one per slice), merge bound."""

    def __init__(self, pixels, n_max, bound=0.0):
        self.pixels = int(pixels)
        self.n_max = n_max
        self.bound = float(bound)


class Plan:
    """Frame plan (vplmc_plan_create, or vplmc_plan_create_coarse with a
    Coarsening and the scene's tree above the cut): host-only layout of every slice."""

    def __init__(self, scene, params, coarsen=None):
        lib = N.load()
        self.n_slices = scene.n_slices
        self.n_clusters = scene.n_clusters
        self.coarse = coarsen is not None
        pt = np.ascontiguousarray(scene.pt_offsets, dtype=np.int32)
        rk = np.ascontiguousarray(scene.rank, dtype=np.int32)
        h = ctypes.c_void_p()
        f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        if coarsen is None:
            cl = np.ascontiguousarray(scene.cl_offsets, dtype=np.int32)
            check(lib.vplmc_plan_create(self.n_slices, f(pt), f(cl), f(rk), self.n_clusters, ctypes.byref(params),
                                        ctypes.byref(h)))
        else:
            left = np.ascontiguousarray(scene.tree_left, dtype=np.int32)
            right = np.ascontiguousarray(scene.tree_right, dtype=np.int32)
            nmax = np.ascontiguousarray(np.broadcast_to(np.asarray(coarsen.n_max), (self.n_slices,)), dtype=np.int32)
            c = N.Coarsen(self.n_clusters, coarsen.pixels, f(left), f(right), f(nmax), coarsen.bound, 0)
            check(lib.vplmc_plan_create_coarse(self.n_slices, f(pt), f(rk), ctypes.byref(c), ctypes.byref(params),
                                               ctypes.byref(h)))
        self.h = h
        sz = ctypes.c_size_t()
        check(lib.vplmc_workspace_size(h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)

    def slice_info(self, s):
        info = N.SliceInfo()
        check(N.load().vplmc_plan_slice(self.h, s, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in N.SliceInfo._fields_}

    def region(self, name):
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        check(N.load().vplmc_plan_region(self.h, N.R[name], ctypes.byref(off), ctypes.byref(nb)))
        return int(off.value), int(nb.value)

    def close(self):
        if self.h:
            N.load().vplmc_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace(plan, device):
    return torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device=device)


def region_view(plan, ws, name, dtype):
    off, nb = plan.region(name)
    return ws[off:off + nb].view(dtype)


def render(ctx, plan, ds, params, ws, radiance=None):
    """One frame (vplmc_render); returns radiance float32 [m, 3] on the device."""
    if radiance is None:
        radiance = torch.empty((ds.m, 3), dtype=torch.float32, device=ws.device)
    check(N.load().vplmc_render(ctx.h, plan.h, ctypes.byref(ds.points_c), ctypes.byref(ds.vpls_c),
                                ctypes.byref(ds.cut_c), _ptr(ds.pt_ids), _ptr(ds.cl_ids), ctypes.byref(params),
                                _ptr(ws), ws.numel(), _ptr(radiance)))
    return radiance


def render_static(ctx, plan, ds, params, radiance=None):
    """One frame on the library's static device workspace (vplmc_render_static):
    no allocation inside the call; returns radiance float32 [m, 3]."""
    if radiance is None:
        radiance = torch.empty((ds.m, 3), dtype=torch.float32, device=ds.pt_ids.device)
    check(N.load().vplmc_render_static(ctx.h, plan.h, ctypes.byref(ds.points_c), ctypes.byref(ds.vpls_c),
                                       ctypes.byref(ds.cut_c), _ptr(ds.pt_ids), _ptr(ds.cl_ids),
                                       ctypes.byref(params), _ptr(radiance)))
    return radiance


def read_stats(ctx, plan, ws):
    S = plan.n_slices
    iters = np.zeros(S, np.int32)
    flags = np.zeros(S, np.int32)
    resid = np.zeros(S, np.float32)
    n2 = np.zeros(S, np.int32)
    f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    check(N.load().vplmc_read_stats(ctx.h, plan.h, _ptr(ws), f(iters), f(flags), f(resid), f(n2)))
    return dict(iters=iters, flags=flags, resid=resid, n2=n2)


def read_counts(ctx, plan, ws):
    """Per-slice n', N1, N2 of the last frame on this workspace (vplmc_read_counts)."""
    S = plan.n_slices
    n, n1, n2 = (np.zeros(S, np.int32) for _ in range(3))
    f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    check(N.load().vplmc_read_counts(ctx.h, plan.h, _ptr(ws), f(n), f(n1), f(n2)))
    return dict(n=n, N1=n1, N2=n2)


def read_totals(ctx, plan, ws):
    """Frame totals (vplmc_read_totals): sampled entries, their shadow rays, the
    coarsening's entry evaluations and its shadow rays."""
    out = np.zeros(4, np.int64)
    check(N.load().vplmc_read_totals(ctx.h, plan.h, _ptr(ws), out.ctypes.data_as(ctypes.c_void_p)))
    return dict(entries=int(out[0]), rays=int(out[1]), coarsen_evals=int(out[2]), coarsen_rays=int(out[3]))


def check_inputs(ctx, plan, ds):
    """vplmc_check_inputs: number of out-of-range point, cluster and member ids."""
    bad = ctypes.c_int64()
    check(N.load().vplmc_check_inputs(ctx.h, plan.h, ds.m, ds.n_vpls, ctypes.byref(ds.cut_c), _ptr(ds.pt_ids),
                                      _ptr(ds.cl_ids), ctypes.byref(bad)))
    return int(bad.value)


def cluster_table(ctx, ds, seed):
    nc = ds.n_clusters
    dev = ds.pt_ids.device
    rep = torch.empty(nc, dtype=torch.int32, device=dev)
    lights = torch.empty((9, nc), dtype=torch.float32, device=dev)
    bbox = torch.empty((6, nc), dtype=torch.float32, device=dev)
    check(N.load().vplmc_cluster_table(ctx.h, ctypes.byref(ds.vpls_c), ctypes.byref(ds.cut_c), int(seed),
                                       _ptr(rep), _ptr(lights), _ptr(bbox)))
    return rep, lights, bbox


def eval_pairs(ctx, ds, lights, point_ids, light_ids, params):
    n = int(point_ids.shape[0])
    out = torch.empty((n, 3), dtype=torch.float32, device=point_ids.device)
    L = lights_struct(lights)
    check(N.load().vplmc_eval_pairs(ctx.h, ctypes.byref(ds.points_c), ctypes.byref(L), n, _ptr(point_ids),
                                    _ptr(light_ids), ctypes.byref(params), _ptr(out)))
    return out


def brute_force(ctx, ds, lights, params, point_ids=None, n_out=None):
    dev = ds.pt_ids.device
    if point_ids is not None:
        n_out = int(point_ids.shape[0])
    elif n_out is None:
        n_out = ds.m
    out = torch.empty((n_out, 3), dtype=torch.float64, device=dev)
    L = lights_struct(lights)
    check(N.load().vplmc_brute_force(ctx.h, ctypes.byref(ds.points_c), ctypes.byref(L), n_out,
                                     _ptr(point_ids), ctypes.byref(params), _ptr(out)))
    return out


# ---- stage calls -----------------------------------------------------------

def stage_pass2(ctx, plan, params, ws):
    """vplmc_stage_pass2: second pass from OMEGA1 and WEIGHTS (already in ws)."""
    check(N.load().vplmc_stage_pass2(ctx.h, plan.h, ctypes.byref(params), _ptr(ws), ws.numel()))


def stage_adm(ctx, plan, params, ds_or_pt_ids, ws, n_points=None, radiance=None):
    """vplmc_stage_adm: completion + sum from OMEGA1/VAL1 (already in ws)."""
    pt_ids = ds_or_pt_ids.pt_ids if hasattr(ds_or_pt_ids, "pt_ids") else ds_or_pt_ids
    n_points = ds_or_pt_ids.m if n_points is None else n_points
    if radiance is None:
        radiance = torch.empty((n_points, 3), dtype=torch.float32, device=ws.device)
    check(N.load().vplmc_stage_adm(ctx.h, plan.h, ctypes.byref(params), _ptr(pt_ids), int(n_points), _ptr(ws),
                                   ws.numel(), _ptr(radiance)))
    return radiance


def stage_reduce(ctx, plan, pt_ids, n_points, ws):
    radiance = torch.empty((n_points, 3), dtype=torch.float32, device=ws.device)
    check(N.load().vplmc_stage_reduce(ctx.h, plan.h, _ptr(pt_ids), int(n_points), _ptr(ws), ws.numel(),
                                      _ptr(radiance)))
    return radiance


def full_matrix(ctx, plan, ds, lights, params, slice_begin, slice_end, cl_ids=None):
    """Every entry of slices [slice_begin, slice_end): float32 [sum m'n', 3]."""
    cl = ds.cl_ids if cl_ids is None else cl_ids
    total = sum(plan.slice_info(s)["m"] * plan.slice_info(s)["n"] for s in range(slice_begin, slice_end))
    out = torch.empty((total, 3), dtype=torch.float32, device=ds.pt_ids.device)
    check(N.load().vplmc_full_matrix(ctx.h, plan.h, ctypes.byref(ds.points_c), _ptr(lights), int(lights.shape[-1]),
                                     _ptr(ds.pt_ids), _ptr(cl), ctypes.byref(params), int(slice_begin),
                                     int(slice_end), _ptr(out)))
    return out


def philox4x64(ctx, key0, key1, ctr):
    """ctr: int64 tensor (n, 4) holding uint64 bit patterns; returns the same layout."""
    n = int(ctr.shape[0])
    out = torch.empty_like(ctr)
    check(N.load().vplmc_philox4x64(ctx.h, key0, key1, _ptr(ctr), n, _ptr(out)))
    return out


def profile_begin(ctx, max_frames):
    check(N.load().vplmc_profile_begin(ctx.h, int(max_frames)))


def profile_end(ctx):
    """Summed ms per phase (dict) over the recorded frames, and the frame count."""
    ms = np.zeros(N.N_PHASES, np.float64)
    fr = np.zeros(1, np.int32)
    check(N.load().vplmc_profile_end(ctx.h, ms.ctypes.data_as(ctypes.c_void_p), fr.ctypes.data_as(ctypes.c_void_p)))
    return dict(zip(N.PHASES, ms.tolist())), int(fr[0])


# ---- global light cut (Sec. 3 step 1, Sec. 6) ---------------------------------

class LightcutPlan:
    """Plan of the global light cut over a full light tree (perm, left, right
    as scenegen.full_light_tree lays it out) for n_samples sample pixels and
    a cut of at most max_cut nodes; validates the tree on the host."""

    def __init__(self, perm, left, right, n_samples, max_cut):
        lib = N.load()
        self.perm = np.ascontiguousarray(perm, dtype=np.int32)
        self._left = np.ascontiguousarray(left, dtype=np.int32)
        self._right = np.ascontiguousarray(right, dtype=np.int32)
        self.n = int(self.perm.shape[0])
        self.n_samples = int(n_samples)
        self.max_cut = int(max_cut)
        f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        tree = N.LightTree(self.n, f(self.perm), f(self._left), f(self._right))
        h = ctypes.c_void_p()
        check(lib.vplmc_lightcut_plan_create(ctypes.byref(tree), self.n_samples, self.max_cut, ctypes.byref(h)))
        self.h = h
        sz = ctypes.c_size_t()
        check(lib.vplmc_lightcut_workspace_size(self.h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)

    def workspace(self, device):
        return torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)

    def close(self):
        if getattr(self, "h", None):
            N.load().vplmc_lightcut_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lightcut(ctx, lplan, ds, sample_ids, eps, r_min, seed, ws, want_rho=False):
    """The global cut (vplmc_lightcut).  Returns device tensors: n_cut (1,),
    cut_nodes (max_cut,), cut_offsets (max_cut + 1,), above_left/right
    (max_cut - 1,) and rho (2 n - 1,) or None; only the first n_cut entries
    of the cut arrays are meaningful."""
    dev = ws.device
    i32 = lambda k: torch.full((max(k, 1),), -1, dtype=torch.int32, device=dev)
    n_cut = i32(1)
    nodes, offs = i32(lplan.max_cut), i32(lplan.max_cut + 1)
    al, ar = i32(lplan.max_cut - 1), i32(lplan.max_cut - 1)
    rho = torch.empty(2 * lplan.n - 1, dtype=torch.float32, device=dev) if want_rho else None
    check(N.load().vplmc_lightcut(ctx.h, lplan.h, ctypes.byref(ds.points_c), ctypes.byref(ds.vpls_c),
                                  _ptr(sample_ids), float(eps), float(r_min), int(seed), _ptr(ws),
                                  int(ws.numel()), _ptr(n_cut), _ptr(nodes), _ptr(offs), _ptr(al), _ptr(ar),
                                  _ptr(rho) if rho is not None else None))
    return dict(n_cut=n_cut, cut_nodes=nodes, cut_offsets=offs, above_left=al, above_right=ar, rho=rho)


# ---- batching: launch shapes, autotuning, captured frames --------------------

def get_tune(plan):
    t = N.Tune()
    check(N.load().vplmc_plan_get_tune(plan.h, ctypes.byref(t)))
    return {"adm_queue": t.adm_queue, "adm_threads": t.adm_threads, "eval_threads": t.eval_threads}


def set_tune(plan, adm_queue=None, adm_threads=None, eval_threads=None):
    cur = get_tune(plan)
    t = N.Tune(cur["adm_queue"] if adm_queue is None else adm_queue,
               cur["adm_threads"] if adm_threads is None else adm_threads,
               cur["eval_threads"] if eval_threads is None else eval_threads, 0)
    check(N.load().vplmc_plan_set_tune(plan.h, ctypes.byref(t)))


def autotune(ctx, plan, ds, params, ws, radiance, reps=2):
    """vplmc_autotune; returns the chosen launch shapes (also left in the plan)."""
    t = N.Tune()
    check(N.load().vplmc_autotune(ctx.h, plan.h, ctypes.byref(ds.points_c), ctypes.byref(ds.vpls_c),
                                  ctypes.byref(ds.cut_c), _ptr(ds.pt_ids), _ptr(ds.cl_ids), ctypes.byref(params),
                                  _ptr(ws), ws.numel(), _ptr(radiance), int(reps), ctypes.byref(t)))
    return {"adm_queue": t.adm_queue, "adm_threads": t.adm_threads, "eval_threads": t.eval_threads}


class Graph:
    """A whole frame captured once (vplmc_graph_create) and replayed by launch().
    The inputs, workspace and radiance tensors must stay alive and in place."""

    def __init__(self, ctx, plan, ds, params, ws, radiance):
        h = ctypes.c_void_p()
        check(N.load().vplmc_graph_create(ctx.h, plan.h, ctypes.byref(ds.points_c), ctypes.byref(ds.vpls_c),
                                          ctypes.byref(ds.cut_c), _ptr(ds.pt_ids), _ptr(ds.cl_ids),
                                          ctypes.byref(params), _ptr(ws), ws.numel(), _ptr(radiance),
                                          ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self._keep = (plan, ds, params, ws, radiance)

    def launch(self):
        check(N.load().vplmc_graph_launch(self.ctx.h, self.h))

    def close(self):
        if self.h:
            N.load().vplmc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned proposal -------------------------------------------------------

def mlp_param_count():
    return N.load().vplmc_mlp_param_count()


def set_proposal(ctx, params):
    """params: device float32 tensor of mlp_param_count() values, or None."""
    check(N.load().vplmc_set_proposal(ctx.h, _ptr(params) if params is not None else None))
    ctx._proposal = params


def mlp_forward(ctx, params, features):
    rows = int(features.shape[0])
    y = torch.empty(rows, dtype=torch.float32, device=features.device)
    check(N.load().vplmc_mlp_forward(ctx.h, _ptr(params), rows, _ptr(features), _ptr(y)))
    return y


def mlp_scratch(rows, device):
    sz = ctypes.c_size_t()
    check(N.load().vplmc_mlp_scratch_size(int(rows), ctypes.byref(sz)))
    return torch.empty(int(sz.value), dtype=torch.uint8, device=device)


def mlp_grad(ctx, params, features, dy, scratch=None):
    rows = int(features.shape[0])
    scratch = mlp_scratch(rows, features.device) if scratch is None else scratch
    g = torch.empty(mlp_param_count(), dtype=torch.float32, device=features.device)
    check(N.load().vplmc_mlp_grad(ctx.h, _ptr(params), rows, _ptr(features), _ptr(dy), _ptr(scratch),
                                  scratch.numel(), _ptr(g)))
    return g


def mlp_adam(ctx, params, grad, m, v, step, lr):
    check(N.load().vplmc_mlp_adam(ctx.h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr)))


def mlp_train_step(ctx, params, m, v, step, lr, features, pstar, group_offsets, scratch, loss):
    rows = int(features.shape[0])
    check(N.load().vplmc_mlp_train_step(ctx.h, _ptr(params), _ptr(m), _ptr(v), int(step), float(lr), rows,
                                        _ptr(features), _ptr(pstar), int(group_offsets.shape[0] - 1),
                                        _ptr(group_offsets), _ptr(scratch), scratch.numel(), _ptr(loss)))


def proposal_targets(ctx, plan, ds, lights, params, ws):
    """p* per (slice, column) in the plan's column layout (device float32)."""
    n = int(plan.region("WEIGHTS")[1] // 4)
    out = torch.empty(n, dtype=torch.float32, device=ws.device)
    check(N.load().vplmc_proposal_targets(ctx.h, plan.h, ctypes.byref(ds.points_c), _ptr(lights), _ptr(ds.pt_ids),
                                          _ptr(ds.cl_ids), ctypes.byref(params), _ptr(ws), ws.numel(), _ptr(out)))
    return out
