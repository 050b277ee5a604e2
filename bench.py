"""Frame benchmark of the sparse-sampling + completion hot path on one MI355X.

One step = one whole frame of the method (cluster table, both sampling
passes, entries with shadow rays, ordering of the samples, ADM completion of every
slice, factorised column sum) on device-resident inputs.  Prints ONE JSON
line.  ``value`` is sampled entries per second of frame time; the frame
time, the pixel RMSE against the brute-force sum over every VPL (sampled
pixels), the per-phase times from HIP events recorded in the timed frames,
the roofline of the dominant kernel and the FP64 CPU oracle timed on a
bounded sample of the same workload are reported beside it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--rate", type=float, default=5.0, help="total sampling rate in percent, split evenly")
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--rmse-pixels", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", default="0.5,1,2,3,4,5,7.5,10",
                    help="total sampling rates (percent) of the plain vs learned fixed-RMSE comparison; empty: none")
    ap.add_argument("--sweep-steps", type=int, default=2)
    ap.add_argument("--eager", action="store_true",
                    help="time eager frames instead of the captured graph (for counter collection)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer 3 times (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


def copy_probe(mib):
    """A plain device copy of known size: what FETCH_SIZE / WRITE_SIZE read for
    it converts the counters of the other kernels to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "copies": 3}), flush=True)


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def frame_times(api, torch, ctx, plan, ds, prm, ws, rad, steps, warmup, eager=False):
    """Mean frame ms of the captured frame graph (or of eager frames) over
    `steps` launches after `warmup` (device-resident inputs); `rad` holds the
    frame afterwards."""
    g = None if eager else api.Graph(ctx, plan, ds, prm, ws, rad)
    launch = g.launch if g else (lambda: api.render(ctx, plan, ds, prm, ws, rad))
    for _ in range(warmup):
        launch()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    if g:
        g.close()
    return e0.elapsed_time(e1) / steps


def interp_ms_at(points, target):
    """Frame ms at pixel RMSE `target` by log-log interpolation over (rmse, ms)
    points of one proposal; None outside their range."""
    pts = sorted(points)
    for (r0, m0), (r1, m1) in zip(pts, pts[1:]):
        if min(r0, r1) <= target <= max(r0, r1) and r0 != r1:
            w = (np.log(target) - np.log(r0)) / (np.log(r1) - np.log(r0))
            return float(np.exp(np.log(m0) + w * (np.log(m1) - np.log(m0))))
    return None


def source_digest():
    """SHA-256 over the completion kernel's sources, line comments and blank
    lines left out: counters taken on other code no longer describe the
    kernel, while an edit of a comment leaves them valid."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels_adm.hip", "vplmc_internal.h"):
        with open(os.path.join(ROOT, "paper_2202_12567_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(workload, ppm):
    """HBM bytes per completion launch from FETCH_SIZE + WRITE_SIZE (rocprofv3
    --pmc, one pass each, scaled by the same counters on a plain copy of known
    size), recorded under profiles/ for this workload, rate and kernel source;
    None when absent or stale."""
    path = os.path.join(ROOT, "profiles", f"k_adm_ell_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("ppm") != ppm or rec.get("source_sha256") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def _oracle_slice(job):
    """One slice through the FP64 oracle (a spawned worker; no GPU)."""
    sub, ppm, seed = job
    from threadpoolctl import threadpool_limits

    from oracle import render as orender
    with threadpool_limits(1):
        _, per = orender.render(sub, orender.Params(seed=seed, pass1_ppm=ppm, pass2_ppm=ppm))
    return sum(r["N1"] + r["N2"] for r in per)


def cpu_baseline(sc, ppm, seed):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: one
    slice per task over the host's cores (spawned processes, one BLAS thread
    each), two tasks per worker."""
    import multiprocessing as mp

    from scenegen import scene_sample
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    step = max(1, sc.n_slices // (2 * workers))
    slices = list(range(0, sc.n_slices, step))[: 2 * workers]
    jobs = [(scene_sample(sc, [s]), ppm, seed) for s in slices]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_slice, jobs[:1])          # worker start-up outside the timing
        t0 = time.perf_counter()
        ent = sum(pool.map(_oracle_slice, jobs, chunksize=1))
        dt = time.perf_counter() - t0
    return {"value": ent / dt, "unit": "entries/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(slices)} of {sc.n_slices} slices (every {step}th; {ent} sampled entries, whole method "
                      f"incl. 100 ADM iterations), {dt:.1f} s wall on {workers} worker processes"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slices would shard across GPUs "
              "with one radiance gather; not implemented here).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2202_12567_amd import api
    from scenegen import make_scene

    dev = torch.device("cuda", 0)
    ppm = int(round(args.rate * 1e4 / 2))
    sc = make_scene(args.workload, args.seed)
    prm = api.default_params(seed=args.seed, pass1_ppm=ppm, pass2_ppm=ppm)
    ctx = api.Context(0)
    ctx.set_occluders(sc.spheres)
    ds = api.DeviceScene(sc, dev)
    plan = api.Plan(sc, prm)
    ws = api.workspace(plan, dev)
    rad = torch.empty((sc.m, 3), dtype=torch.float32, device=dev)
    # the proposal network trained on scenes of this workload's shape, else the default one
    weights_path = os.path.join(ROOT, "paper_2202_12567_amd", f"proposal_mlp_{args.workload}.npy")
    if not os.path.exists(weights_path):
        weights_path = os.path.join(ROOT, "paper_2202_12567_amd", "proposal_mlp.npy")
    proposal = None
    if os.path.exists(weights_path):
        proposal = torch.as_tensor(np.load(weights_path)).to(dev)
        api.set_proposal(ctx, proposal)

    # the frame as a captured graph (or eager calls on the library's stream):
    # W untimed launches, then exactly K timed ones, an event after each
    graph = None if args.eager else api.Graph(ctx, plan, ds, prm, ws, rad)
    frame = graph.launch if graph else (lambda: api.render(ctx, plan, ds, prm, ws, rad))
    progress(f"{args.workload}: {sc.n_slices} slices, workspace {plan.workspace_bytes / 1e9:.1f} GB")
    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()
    progress("warm-up done")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for k in range(args.steps):
        frame()
        ev[k + 1].record()
    torch.cuda.synchronize()
    per_frame = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    ms_median = float(np.median(per_frame))
    if graph:
        graph.close()
    progress(f"timed {args.steps} frames: {ms:.3f} ms per frame")

    # phase times from HIP events around each phase (eager frames of the same plan)
    api.profile_begin(ctx, args.steps)
    for _ in range(args.steps):
        api.render(ctx, plan, ds, prm, ws, rad)
    torch.cuda.synchronize()
    phase_ms, frames = api.profile_end(ctx)
    progress("phase times done")
    phase_ms = {k: v / max(frames, 1) for k, v in phase_ms.items()}
    eager_ms = sum(phase_ms.values())

    st = api.read_stats(ctx, plan, ws)
    infos = [plan.slice_info(s) for s in range(sc.n_slices)]
    N1 = np.array([i["N1"] for i in infos], np.int64)
    n2 = st["n2"].astype(np.int64)
    entries = int(N1.sum() + n2.sum())
    q = np.array([i["q"] for i in infos], np.int64)
    iters = st["iters"].astype(np.int64)
    omega = N1 + n2
    sample_iters = int((omega * iters).sum())

    # pixel RMSE against the brute-force sum over every VPL, on sampled pixels
    rng = np.random.default_rng(12345)
    pid = np.sort(rng.choice(sc.m, min(args.rmse_pixels, sc.m), replace=False)).astype(np.int32)
    pid_t = torch.as_tensor(pid, device=dev)
    ref = api.brute_force(ctx, ds, ds.vpl, prm, point_ids=pid_t)
    rep, lights, _ = api.cluster_table(ctx, ds, args.seed)
    cut_ref = api.brute_force(ctx, ds, lights, prm, point_ids=pid_t)
    got = rad[pid_t.long()].double()
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    rmse_full = rel(got, ref)
    rmse_cut = rel(got, cut_ref)
    cut_vs_full = rel(cut_ref, ref)
    progress("reference sums done")

    # roofline of the dominant kernel (the completion, one launch per frame):
    # algorithmic HBM bytes = 16 B (row index + RGB) per sampled entry per
    # iteration + 4 q (6 m' + 18 n') B of factor state (X, U, L and Y, V, P
    # read and written) per slice per iteration; FP32 work = 18 q flop per
    # sampled entry per iteration
    t_adm = phase_ms["adm"] * 1e-3
    m_s = np.array([i["m"] for i in infos], np.int64)
    n_s = np.array([i["n"] for i in infos], np.int64)
    sample_bytes = 16.0 * sample_iters
    state_bytes = float((4 * q * (6 * m_s + 18 * n_s) * iters).sum())
    adm_bytes = sample_bytes + state_bytes
    adm_flops = float((18 * q * omega * iters).sum())
    achieved = adm_bytes / t_adm / 1e9
    all_ell = all(i["adm_in_lds"] for i in infos)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, ppm) if all_ell else None,
            "kernel": "k_adm_ell" if all_ell else "k_adm_ell + k_adm",
            "kernel_ms": round(phase_ms["adm"], 3),
            "algorithmic_bytes": {"samples": sample_bytes, "factor_state": state_bytes},
            "fp32_tflops": round(adm_flops / t_adm / 1e12, 2),
            "fp32_frac": round(adm_flops / t_adm / 1e12 / FP32_PEAK_TFLOPS, 4)}
    dominant = max(phase_ms, key=phase_ms.get)

    # learned proposal at the same rate, and the plain vs learned sweep
    learned = None
    fixed = None
    if proposal is not None:
        prm_l = api.default_params(seed=args.seed, pass1_ppm=ppm, pass2_ppm=ppm, learned=True)
        rad_l = torch.empty_like(rad)
        ms_l = frame_times(api, torch, ctx, plan, ds, prm_l, ws, rad_l, args.steps, 1, args.eager)
        st_l = api.read_stats(ctx, plan, ws)
        rmse_l = rel(rad_l[pid_t.long()].double(), ref)
        learned = {"weights": os.path.basename(weights_path), "frame_ms": round(ms_l, 3),
                   "pixel_rmse_vs_full_sum": round(rmse_l, 5),
                   "fallback_slices": int(((st_l["flags"] & 8) != 0).sum()),
                   "sampled_entries_per_frame": int(N1.sum() + st_l["n2"].astype(np.int64).sum())}
        rates = [float(x) for x in args.sweep.split(",") if x.strip()]
        if rates:
            pts = {"plain": [], "learned": []}
            rows = []
            for r in rates:
                pr = int(round(r * 1e4 / 2))
                pl = api.Plan(sc, api.default_params(seed=args.seed, pass1_ppm=pr, pass2_ppm=pr))
                wsr = api.workspace(pl, dev)
                row = {"rate_pct": r}
                for name, flag in (("plain", False), ("learned", True)):
                    pp = api.default_params(seed=args.seed, pass1_ppm=pr, pass2_ppm=pr, learned=flag)
                    msr = frame_times(api, torch, ctx, pl, ds, pp, wsr, rad_l, args.sweep_steps, 1, args.eager)
                    er = rel(rad_l[pid_t.long()].double(), ref)
                    pts[name].append((er, msr))
                    row[name] = {"frame_ms": round(msr, 3), "pixel_rmse": round(er, 5)}
                rows.append(row)
                progress(f"sweep {r}%: plain {row['plain']['frame_ms']} ms, learned {row['learned']['frame_ms']} ms")
                del wsr
                pl.close()
            target = rmse_full
            ms_plain_t = interp_ms_at(pts["plain"], target)
            ms_learned_t = interp_ms_at(pts["learned"], target)

            def first_meeting(name):
                ok = [(r, p) for r, p in zip(rates, pts[name]) if p[0] <= target * (1 + 1e-9)]
                return None if not ok else {"rate_pct": ok[0][0], "frame_ms": round(ok[0][1][1], 3)}

            fixed = {"target_pixel_rmse": round(target, 5),
                     "plain_at_smallest_rate": first_meeting("plain"),
                     "learned_at_smallest_rate": first_meeting("learned"),
                     "plain_ms_interpolated": None if ms_plain_t is None else round(ms_plain_t, 3),
                     "learned_ms_interpolated": None if ms_learned_t is None else round(ms_learned_t, 3),
                     "learned_speedup_interpolated": None if not (ms_plain_t and ms_learned_t)
                     else round(ms_plain_t / ms_learned_t, 3),
                     "sweep": rows}

    out = {
        "metric": "frame ms at fixed pixel RMSE vs full sum; sampled entries/s; plain vs learned",
        "value": round(entries / (ms * 1e-3), 1),
        "unit": "sampled entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {sc.m} points, {sc.n} VPLs, {sc.n_clusters}-cluster cut, "
                               f"{sc.n_slices} slices, rank {int(q.max())}, {args.rate:g}% sampling "
                               f"({ppm} + {ppm} ppm), {len(sc.spheres['r'])} spheres",
                   "seed": args.seed, "proposal": "plain"},
        "frame_ms": round(ms, 3),
        "frame_ms_median": round(ms_median, 3),
        "timing": ("eager frames" if args.eager else "captured frame graph (vplmc_graph_create)")
                  + ", HIP events per launch; phase_ms from eager frames",
        "eager_frame_ms_sum_of_phases": round(eager_ms, 3),
        "sampled_entries_per_frame": entries,
        "pixel_rmse_vs_full_sum": round(rmse_full, 5),
        "pixel_rmse_vs_cut_sum": round(rmse_cut, 5),
        "cut_sum_rmse_vs_full_sum": round(cut_vs_full, 5),
        "rmse_pixels": int(pid.shape[0]),
        "adm_iterations_mean": float(iters.mean()),
        "phase_ms": {k: round(v, 3) for k, v in phase_ms.items()},
        "dominant_phase": dominant,
        "roofline": roof,
        "learned": learned,
        "fixed_rmse": fixed,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, ppm, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
