"""Frame benchmark of the sparse-sampling + completion hot path on one MI355X.

One step = one whole frame of the method (cluster table, per-slice light
coarsening, both sampling passes, entries with shadow rays, ordering of the
samples, ADM completion of every slice, factorised column sum) on
device-resident inputs.  The default workload is the 1920 x 1080 frame
(300,000 VPLs, 16,384-cluster cut, 3,069 slices) with every slice coarsened
to at most 512 columns from 32,768 row draws, rank 16, second pass at 1% of
the coarsened slice matrix.  Prints ONE JSON line.  ``value`` is sampled entries per second of frame time; the frame
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
    ap.add_argument("--workload", default="frame")
    ap.add_argument("--rate", type=float, default=None,
                    help="sampling rate in percent: of the second pass with coarsening (default 1), else the total, "
                         "split evenly between the passes (default 5)")
    ap.add_argument("--coarsen", default=None,
                    help="K:n_max: coarsen every slice from K row draws to at most n_max columns; 'none' to keep "
                         "the cut (default 32768:512 for the frame workload, none otherwise)")
    ap.add_argument("--rank", type=int, default=None, help="rank of every slice (default 16 with coarsening)")
    ap.add_argument("--seed", type=int, default=None, help="scene seed (frame 41, mid 11, batch 21)")
    ap.add_argument("--rmse-pixels", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", default="0.5,1,2,3,5,7.5,10",
                    help="total sampling rates (percent) of the plain vs learned fixed-RMSE comparison; empty: none")
    ap.add_argument("--sweep-steps", type=int, default=1)
    ap.add_argument("--lightcut", default="0.02:16384:8192",
                    help="EPS:MAX_CUT:SAMPLES of the global light cut timed over every VPL (Sec. 3 step 1); "
                         "'none' to skip")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of running vplmc_autotune before the timing")
    ap.add_argument("--launch-shape", default=None, metavar="QUEUE:THREADS:EVAL",
                    help="use these launch shapes (completion work queue 0/1, completion threads, entry threads) "
                         "instead of the autotuner's")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the completion variants and the rank sweep at the headline rate")
    ap.add_argument("--eager", action="store_true",
                    help="time eager frames instead of the captured graph (for counter collection)")
    ap.add_argument("--write-traffic", nargs=4, metavar="CSV", default=None,
                    help="write the completion's traffic record from rocprofv3 --pmc CSVs (FETCH_SIZE, WRITE_SIZE "
                         "of this benchmark, then of --copy-probe 1024) and exit")
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
    for f in ("kernels_adm.hip", "adm_common.h", "vplmc_internal.h"):
        with open(os.path.join(ROOT, "paper_2202_12567_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(workload, ppm, coarsen="none", rank=0, adm_threads=1024, adm_queue=0):
    """HBM bytes per completion launch from FETCH_SIZE + WRITE_SIZE (rocprofv3
    --pmc, one pass each, scaled by the same counters on a plain copy of known
    size), recorded under profiles/ for this workload, rate, coarsening, rank,
    launch shape and kernel source; None when absent or stale."""
    path = os.path.join(ROOT, "profiles", f"k_adm_ell_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("ppm") != ppm or rec.get("source_sha256") != source_digest()
            or rec.get("coarsen", "none") != coarsen or rec.get("rank", 0) != rank
            or rec.get("adm_threads", 1024) != adm_threads or rec.get("adm_queue", 0) != adm_queue):
        return None
    return rec.get("bytes_per_launch")


def _pmc_per_dispatch(path, kernel_prefix, counter):
    """Mean value of `counter` over the dispatches of kernels whose name
    contains kernel_prefix, from a rocprofv3 --pmc counter_collection CSV."""
    import csv
    vals = {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter or kernel_prefix not in row.get("Kernel_Name", ""):
                continue
            key = row.get("Dispatch_Id") or row.get("Correlation_Id")
            vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel_prefix} in {path}")
    return sum(vals.values()) / len(vals), len(vals)


def write_traffic_record(args, csvs):
    """profiles/k_adm_ell_<workload>_traffic.json from four rocprofv3 --pmc
    CSVs: FETCH_SIZE and WRITE_SIZE of the benchmark, then of --copy-probe."""
    f_csv, w_csv, cf_csv, cw_csv = csvs
    shape = tuple(int(v) for v in (args.launch_shape or "0:1024:256").split(":"))
    fetch, nf = _pmc_per_dispatch(f_csv, "::k_adm_ell<", "FETCH_SIZE")
    write, nw = _pmc_per_dispatch(w_csv, "::k_adm_ell<", "WRITE_SIZE")
    probe = 1 << 30
    # the probe's device-to-device copies (not the fill that initialises the source)
    cfetch, _ = _pmc_per_dispatch(cf_csv, "copyBuffer", "FETCH_SIZE")
    cwrite, _ = _pmc_per_dispatch(cw_csv, "copyBuffer", "WRITE_SIZE")
    ff = probe / 1024.0 / cfetch
    wf = probe / 1024.0 / cwrite
    rd = int(round(fetch * 1024 * ff))
    wr = int(round(write * 1024 * wf))
    cspec = args.coarsen if args.coarsen is not None else ("32768:512" if args.workload == "frame" else "none")
    rate = args.rate if args.rate is not None else (1.0 if cspec != "none" else 5.0)
    ppm = int(round(rate * 1e4)) if cspec != "none" else int(round(rate * 1e4 / 2))
    rank = args.rank if args.rank is not None else (16 if cspec != "none" else 0)
    wl = "" if args.workload == "frame" else f"--workload {args.workload} --coarsen {cspec} --rank {rank} "
    rec = {"kernel": "k_adm_ell", "workload": args.workload, "ppm": ppm, "coarsen": cspec, "rank": rank,
           "adm_threads": shape[1], "adm_queue": shape[0],   # the shape the counter runs used
           "source_sha256": source_digest(), "fetch_size_kib_per_dispatch": round(fetch, 1),
           "write_size_kib_per_dispatch": round(write, 1), "dispatches": [nf, nw], "copy_probe_bytes": probe,
           "copy_fetch_size_kib": round(cfetch, 1), "copy_write_size_kib": round(cwrite, 1),
           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4), "bytes_per_launch": rd + wr,
           "read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
           "commands": [f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {c} -d <out> -o <name> --output-format csv "
                        f"-- python3 /root/repo/bench.py {wl}--eager --steps 1 --warmup 0 --sweep \"\" --no-cpu-baseline "
                        f"--no-variants --lightcut none --launch-shape {':'.join(map(str, shape))}"
                        for c in ("FETCH_SIZE", "WRITE_SIZE")]
           + [f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {c} -d <out> -o <name> --output-format csv "
              f"-- python3 /root/repo/bench.py --copy-probe 1024" for c in ("FETCH_SIZE", "WRITE_SIZE")]}
    path = os.path.join(ROOT, "profiles", f"k_adm_ell_{args.workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec), flush=True)


_WORKER = {}


def _worker_scene(workload, seed, rank, coarsen):
    """The scene (and the coarsening's node table) of a worker process, built once."""
    key = (workload, seed, rank, coarsen is not None)
    if key not in _WORKER:
        from oracle import coarsen as ocoarsen
        from scenegen import make_scene, supported_rank
        sc = make_scene(workload, seed)
        if rank:
            sc.rank = supported_rank(rank, np.diff(sc.pt_offsets))
        _WORKER[key] = (sc, ocoarsen.scene_table(sc, seed) if coarsen else None)
    return _WORKER[key]


def _warm(job):
    """Builds the worker's scene outside the timed region; the pause keeps every
    worker on one warm-up task."""
    _worker_scene(*job)
    time.sleep(2.0)
    return 0


def _oracle_slice(job):
    """One slice through the FP64 oracle (a spawned worker; no GPU): the plain
    frame's slice, or the coarsened slice (Sec. 4) when a coarsening is given.
    Returns its sampled entries (first + second pass)."""
    workload, seed, s, ppm1, ppm2, rank, coarsen = job
    from threadpoolctl import threadpool_limits

    from oracle import coarsen as ocoarsen
    from oracle import render as orender
    from scenegen import scene_sample
    sc, table = _worker_scene(workload, seed, rank, coarsen)
    prm = orender.Params(seed=seed, pass1_ppm=ppm1, pass2_ppm=ppm2)
    with threadpool_limits(1):
        if coarsen:
            r = ocoarsen.render_slice_coarsened(sc, table, s, prm, ocoarsen.CoarsenParams(pixels=coarsen[0]),
                                                coarsen[1])
            return r["N1"] + r["N2"]
        _, per = orender.render(scene_sample(sc, [s]), prm)
    return sum(r["N1"] + r["N2"] for r in per)


def cpu_baseline(workload, seed, n_slices, ppm1, ppm2, rank, coarsen):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: one
    slice per task (evenly spaced over the frame) over the host's cores
    (spawned processes, one BLAS thread each)."""
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    # a coarsened 1080p slice takes about a minute of one core: one per worker
    tasks = workers if coarsen else 2 * workers
    step = max(1, n_slices // tasks)
    slices = list(range(0, n_slices, step))[:tasks]
    jobs = [(workload, seed, s, ppm1, ppm2, rank, coarsen) for s in slices]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_warm, [(workload, seed, rank, coarsen)] * workers, chunksize=1)   # start-up outside the timing
        t0 = time.perf_counter()
        ent = sum(pool.map(_oracle_slice, jobs, chunksize=1))
        dt = time.perf_counter() - t0
    what = ("coarsening, both passes, 100 ADM iterations, sum" if coarsen
            else "both passes, 100 ADM iterations, sum")
    return {"value": ent / dt, "unit": "sampled entries/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(slices)} of {n_slices} slices (every {step}th; {ent} sampled entries, whole method: "
                      f"{what}), {dt:.1f} s wall on {workers} worker processes"}


SEEDS = {"frame": 41, "mid": 11, "batch": 21, "tiny": 1, "tri": 1, "trimid": 11}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.write_traffic:
        write_traffic_record(args, args.write_traffic)
        return
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slices would shard across GPUs "
              "with one radiance gather; not implemented here).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2202_12567_amd import api
    from scenegen import make_scene, supported_rank

    dev = torch.device("cuda", 0)
    seed = args.seed if args.seed is not None else SEEDS.get(args.workload, 1)
    cspec = args.coarsen if args.coarsen is not None else ("32768:512" if args.workload == "frame" else "none")
    coarsen = None if cspec == "none" else tuple(int(v) for v in cspec.split(":"))
    rank = args.rank if args.rank is not None else (16 if coarsen else 0)
    rate = args.rate if args.rate is not None else (1.0 if coarsen else 5.0)

    def ppms(r):
        """(first, second) pass ppm of a rate in percent"""
        return (0, int(round(r * 1e4))) if coarsen else (int(round(r * 1e4 / 2)),) * 2

    def make_plan(p):
        return api.Plan(sc, p, api.Coarsening(*coarsen) if coarsen else None)

    ppm1, ppm2 = ppms(rate)
    sc = make_scene(args.workload, seed)
    if rank:
        sc.rank = supported_rank(rank, np.diff(sc.pt_offsets))
    prm = api.default_params(seed=seed, pass1_ppm=ppm1, pass2_ppm=ppm2)
    ctx = api.Context(0)
    ctx.set_occluders(sc.spheres)
    ds = api.DeviceScene(sc, dev)
    plan = make_plan(prm)
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

    # launch shapes (completion queue and workgroup size, entry workgroup size)
    # chosen by the library's autotuner on these inputs, before any timing
    if args.launch_shape:
        qv, tv, ev = (int(v) for v in args.launch_shape.split(":"))
        api.set_tune(plan, adm_queue=qv, adm_threads=tv, eval_threads=ev)
        tune = api.get_tune(plan)
    elif not args.no_autotune:
        tune = api.autotune(ctx, plan, ds, prm, ws, rad, reps=2)
    else:
        tune = api.get_tune(plan)
    progress(f"launch shapes: {tune}")
    plain_plan = make_plan

    def make_plan(p):          # the other plans of this run take the same shapes
        pl = plain_plan(p)
        api.set_tune(pl, **tune)
        return pl

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
    n_prof = max(1, min(2, args.steps))
    api.profile_begin(ctx, n_prof)
    for _ in range(n_prof):
        api.render(ctx, plan, ds, prm, ws, rad)
    torch.cuda.synchronize()
    phase_ms, frames = api.profile_end(ctx)
    progress("phase times done")
    phase_ms = {k: v / max(frames, 1) for k, v in phase_ms.items()}
    eager_ms = sum(phase_ms.values())

    st = api.read_stats(ctx, plan, ws)
    cnt = api.read_counts(ctx, plan, ws)
    tot = api.read_totals(ctx, plan, ws)
    infos = [plan.slice_info(s) for s in range(sc.n_slices)]
    N1 = cnt["N1"].astype(np.int64)
    n2 = st["n2"].astype(np.int64)
    entries = int(N1.sum() + n2.sum())
    q = np.array([i["q"] for i in infos], np.int64)
    iters = st["iters"].astype(np.int64)
    omega = N1 + n2
    sample_iters = int((omega * iters).sum())
    m_s = np.array([i["m"] for i in infos], np.int64)
    n_s = cnt["n"].astype(np.int64)
    matrix_entries = int((m_s * n_s).sum())

    # pixel RMSE against the brute-force sum over every VPL, on sampled pixels
    rng = np.random.default_rng(12345)
    pid = np.sort(rng.choice(sc.m, min(args.rmse_pixels, sc.m), replace=False)).astype(np.int32)
    pid_t = torch.as_tensor(pid, device=dev)
    ref = api.brute_force(ctx, ds, ds.vpl, prm, point_ids=pid_t)
    rep, lights, _ = api.cluster_table(ctx, ds, seed)
    cut_ref = api.brute_force(ctx, ds, lights, prm, point_ids=pid_t)
    got = rad[pid_t.long()].double()
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    rmse_full = rel(got, ref)
    rmse_cut = rel(got, cut_ref)
    cut_vs_full = rel(cut_ref, ref)
    progress("reference sums done")

    # roofline of the dominant kernel (the completion, one launch per rank
    # group): algorithmic HBM bytes = 16 B (row index + RGB) per sampled entry
    # per iteration + 4 q (6 m' + 18 n') B of factor state (X, U, L and Y, V, P
    # read and written) per slice per iteration; FP32 work = 18 q flop per
    # sampled entry per iteration (q the slice's rank)
    t_adm = phase_ms["adm"] * 1e-3
    sample_bytes = 16.0 * sample_iters
    state_bytes = float((4 * q * (6 * m_s + 18 * n_s) * iters).sum())
    adm_bytes = sample_bytes + state_bytes
    adm_flops = float((18 * q * omega * iters).sum())
    achieved = adm_bytes / t_adm / 1e9
    all_ell = all(i["adm_in_lds"] for i in infos)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, ppm2 if coarsen else ppm1, cspec, rank, tune["adm_threads"],
                                        tune["adm_queue"]) if all_ell else None,
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
        prm_l = api.default_params(seed=seed, pass1_ppm=ppm1, pass2_ppm=ppm2, learned=True)
        rad_l = torch.empty_like(rad)
        ms_l = frame_times(api, torch, ctx, plan, ds, prm_l, ws, rad_l, min(args.steps, 3), 1, args.eager)
        st_l = api.read_stats(ctx, plan, ws)
        rmse_l = rel(rad_l[pid_t.long()].double(), ref)
        learned = {"weights": os.path.basename(weights_path), "frame_ms": round(ms_l, 3),
                   "pixel_rmse_vs_full_sum": round(rmse_l, 5),
                   "fallback_slices": int(((st_l["flags"] & 8) != 0).sum()),
                   "sampled_entries_per_frame": int(N1.sum() + st_l["n2"].astype(np.int64).sum())}
        rates = [float(x) for x in args.sweep.split(",") if x.strip()]
        if rates:
            ws = None                     # the headline workspace is not needed past this point
            torch.cuda.empty_cache()
            # the baselines that separate what the network adds from what a
            # flatter second pass alone gives: the uniform density and the
            # density g(j) + 3 mean g (the mix of the network's training target)
            kinds = (("plain", False, 0.0), ("learned", True, 0.0), ("uniform", False, float("inf")),
                     ("g_plus_3_mean_g", False, 3.0))
            pts = {name: [] for name, _, _ in kinds}
            rows = []
            for r in rates:
                p1, p2 = ppms(r)
                pl = make_plan(api.default_params(seed=seed, pass1_ppm=p1, pass2_ppm=p2))
                wsr = api.workspace(pl, dev)
                row = {"rate_pct": r}
                for name, flag, mix in kinds:
                    pp = api.default_params(seed=seed, pass1_ppm=p1, pass2_ppm=p2, learned=flag, pass2_mix=mix)
                    msr = frame_times(api, torch, ctx, pl, ds, pp, wsr, rad_l, args.sweep_steps, 1, args.eager)
                    er = rel(rad_l[pid_t.long()].double(), ref)
                    pts[name].append((er, msr))
                    row[name] = {"frame_ms": round(msr, 3), "pixel_rmse": round(er, 5)}
                rows.append(row)
                progress(f"sweep {r}%: " + ", ".join(f"{k} {row[k]['frame_ms']} ms / {row[k]['pixel_rmse']}"
                                                     for k, _, _ in kinds))
                del wsr
                pl.close()
                torch.cuda.empty_cache()
            # the plain method's error at 5% is the target (the highest rate the configuration names)
            ref_rate = 5.0 if 5.0 in rates else rates[-1]
            target = pts["plain"][rates.index(ref_rate)][0]
            ms_plain_t = interp_ms_at(pts["plain"], target)
            ms_learned_t = interp_ms_at(pts["learned"], target)

            def first_meeting(name):
                ok = [(r, p) for r, p in zip(rates, pts[name]) if p[0] <= target * (1 + 1e-9)]
                return None if not ok else {"rate_pct": ok[0][0], "frame_ms": round(ok[0][1][1], 3)}

            fixed = {"target": f"plain pixel RMSE at {ref_rate:g}%",
                     "target_pixel_rmse": round(target, 5),
                     "plain_at_smallest_rate": first_meeting("plain"),
                     "learned_at_smallest_rate": first_meeting("learned"),
                     "baselines_at_smallest_rate": {k: first_meeting(k) for k in ("uniform", "g_plus_3_mean_g")},
                     "baselines_ms_interpolated": {k: (None if (v := interp_ms_at(pts[k], target)) is None
                                                       else round(v, 3)) for k in ("uniform", "g_plus_3_mean_g")},
                     "plain_ms_interpolated": None if ms_plain_t is None else round(ms_plain_t, 3),
                     "learned_ms_interpolated": None if ms_learned_t is None else round(ms_learned_t, 3),
                     "learned_speedup_interpolated": None if not (ms_plain_t and ms_learned_t)
                     else round(ms_plain_t / ms_learned_t, 3),
                     "sweep": rows}

    # completion variants (ADM, ADM without non-negativity, masked ALS) and
    # ranks 8 / 16 / 32 at the headline rate: one graph frame each
    variants = None
    if not args.no_variants:
        ws = None
        torch.cuda.empty_cache()
        rad_v = torch.empty_like(rad)
        variants = {"completion": [], "rank": []}
        for name, kw in (("adm", {}), ("adm_without_nonnegativity", dict(no_nonneg=True)),
                         ("masked_als", dict(als=True))):
            pv = api.default_params(seed=seed, pass1_ppm=ppm1, pass2_ppm=ppm2, **kw)
            pl = make_plan(pv)
            wsv = api.workspace(pl, dev)
            msv = frame_times(api, torch, ctx, pl, ds, pv, wsv, rad_v, 1, 1, args.eager)
            variants["completion"].append({"method": name, "frame_ms": round(msv, 3),
                                           "pixel_rmse": round(rel(rad_v[pid_t.long()].double(), ref), 5)})
            progress(f"variant {name}: {msv:.1f} ms")
            del wsv
            pl.close()
            torch.cuda.empty_cache()
        rank0 = sc.rank.copy()
        for qv in (8, 16, 32):
            sc.rank = supported_rank(qv, np.diff(sc.pt_offsets))
            pv = api.default_params(seed=seed, pass1_ppm=ppm1, pass2_ppm=ppm2)
            pl = make_plan(pv)
            wsv = api.workspace(pl, dev)
            msv = frame_times(api, torch, ctx, pl, ds, pv, wsv, rad_v, 1, 1, args.eager)
            variants["rank"].append({"rank": qv, "frame_ms": round(msv, 3),
                                     "pixel_rmse": round(rel(rad_v[pid_t.long()].double(), ref), 5)})
            progress(f"rank {qv}: {msv:.1f} ms")
            del wsv
            pl.close()
            torch.cuda.empty_cache()
        sc.rank = rank0

    # the global light cut over the full light tree of every VPL (Sec. 3 step
    # 1, Sec. 6): the tree is an input (built on the host, outside the timing);
    # the call uploads it, builds the node table and runs the level-by-level
    # split test on the GPU
    lightcut = None
    if args.lightcut != "none":
        from scenegen import full_light_tree
        lc_eps, lc_cap, lc_S = args.lightcut.split(":")
        lc_eps, lc_cap, lc_S = float(lc_eps), int(lc_cap), min(int(lc_S), sc.m)
        ws = None
        torch.cuda.empty_cache()
        perm, left, right = full_light_tree(np.stack([sc.vpls["x"], sc.vpls["y"], sc.vpls["z"]], 1))
        lp = api.LightcutPlan(perm, left, right, lc_S, lc_cap)
        wsl = lp.workspace(dev)
        sid = torch.as_tensor(np.sort(np.random.default_rng(seed).choice(sc.m, lc_S, replace=False)).astype(np.int32),
                              device=dev)
        run = lambda: api.lightcut(ctx, lp, ds, sid, lc_eps, prm.r_min, seed, wsl, want_rho=True)
        out_lc = run()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 10))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for k in range(reps):
            out_lc = run()
            ev[k + 1].record()
        torch.cuda.synchronize()
        lc_ms = ev[0].elapsed_time(ev[-1]) / reps
        ng = int(out_lc["n_cut"].item())
        rho_lc = out_lc["rho"].cpu().numpy()
        n_tested = int((rho_lc >= 0).sum())
        lightcut = {"vpls": sc.n, "samples": lc_S, "eps": lc_eps, "max_cut": lc_cap, "cut_nodes": ng,
                    "tested_nodes": n_tested, "ms": round(lc_ms, 3),
                    "bound_evaluations": n_tested * lc_S,
                    "estimate_entries": 2 * (ng - 1) * lc_S,
                    "timing": f"HIP events around {reps} calls (tree upload, node table, levels, output)"}
        progress(f"global light cut: {ng} nodes in {lc_ms:.2f} ms")
        del wsl
        lp.close()
        torch.cuda.empty_cache()

    if coarsen:
        rate_txt = (f"every slice coarsened from {coarsen[0]} row draws to at most {coarsen[1]} of the "
                    f"{sc.n_clusters}-cluster cut's nodes, second pass {rate:g}% ({ppm2} ppm) of the coarsened "
                    f"slice matrix")
    else:
        rate_txt = f"{sc.n_clusters}-cluster cut, {rate:g}% sampling ({ppm1} + {ppm2} ppm)"
    out = {
        "metric": "frame ms at fixed pixel RMSE vs full sum; sampled entries/s; plain vs learned",
        "value": round(entries / (ms * 1e-3), 1),
        "unit": "sampled entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {sc.m} points, {sc.n} VPLs, {sc.n_slices} slices, {rate_txt}, "
                               f"rank {int(q.min())}-{int(q.max())}, "
                               + (f"{len(sc.spheres['tri'])} triangles (SBVH), instant-radiosity VPLs" if "tri" in sc.spheres
                                  else f"{len(sc.spheres['r'])} spheres"),
                   "seed": seed, "proposal": "plain"},
        "frame_ms": round(ms, 3),
        "frame_ms_median": round(ms_median, 3),
        "launch_shapes": dict(tune, autotuned=not (args.no_autotune or args.launch_shape)),
        "timing": ("eager frames" if args.eager else "captured frame graph (vplmc_graph_create)")
                  + ", HIP events per launch; phase_ms from eager frames",
        "eager_frame_ms_sum_of_phases": round(eager_ms, 3),
        "sampled_entries_per_frame": entries,
        "first_pass_entries_per_frame": int(N1.sum()),
        "sampled_fraction_of_slice_matrices": round(entries / matrix_entries, 5),
        "columns_per_slice": {"min": int(n_s.min()), "mean": round(float(n_s.mean()), 1), "max": int(n_s.max())},
        # shadow rays (sampled entries whose point and light face each other) over
        # the entry phases' time; the coarsening's unit-intensity evaluations over its phase
        "rays": {"entry_rays_per_frame": tot["rays"],
                 "entry_rays_per_s": round(tot["rays"] / ((phase_ms["eval1"] + phase_ms["eval2"]) * 1e-3), 1),
                 "coarsen_evals_per_frame": tot["coarsen_evals"], "coarsen_rays_per_frame": tot["coarsen_rays"],
                 "coarsen_rays_per_s": round(tot["coarsen_rays"] / max(phase_ms["coarsen"] * 1e-3, 1e-9), 1)},
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
        "variants": variants,
        "global_lightcut": lightcut,
    }
    if not args.no_cpu_baseline:
        progress("oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(args.workload, seed, sc.n_slices, ppm1, ppm2, rank, coarsen)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
