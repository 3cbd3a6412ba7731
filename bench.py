"""Throughput of the coupled step on one MI355X.

Workload (default): 256^3 periodic box, two components at 0.35 +- 0.01 each
(50:50), g = 0.08, tau = 1, 4806 spheres of radius 5 (volume fraction 0.15)
at seeded random positions, neutral wettability, particle density 1, FP32.
A step is one whole time step of the method (densities, virtual fluid,
Shan-Chen force, collision, streaming with moving bounce-back, link and
virtual-fluid force sums, pair forces, leap-frog, map update with covering
and refilling).  Inputs are resident in HBM when the timed region starts.

Prints one JSON line: MLUPS over all lattice sites (and MFLUPS over the fluid
sites), the roofline of the dominant kernel (the sweep that collides and
streams the populations, timed with HIP events on its stream inside the
timed region), set beside the bandwidth a plain elementwise copy reaches on
the same device, and the FP64 oracle timed on the host cores on a bounded
sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (2-comp D3Q19 + spheres) at 256^3 vs HBM roofline; jobs/hour + p99 latency"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_site(precision):
    """Populations read once and written once: 2 components x 19 x (2, 4 or 8) B x 2."""
    ts = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[precision]
    return 2 * 19 * ts * 2


def measured_traffic(kernel, precision, tile):
    """HBM bytes per launch of the dominant sweep from the committed counter
    summary of that sweep, or None when its sources changed since the
    counters were taken"""
    import hashlib
    import re
    name = {("twopass", "fp32"): "bijel256_collide_traffic.md",
            ("fused", "fp32"): "bijel256_fused_traffic.md"}.get((kernel, precision))
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_files = re.search(r"source-sha256 \(([^)]*)\): ([0-9a-f]{64})", text)
    m_bytes = re.search(r"traffic-bytes-per-launch: (\d+)", text)
    m_tile = re.search(r"tile: (\S+)", text)
    if not m_files or not m_bytes or (m_tile and m_tile.group(1) != tile):
        return None
    h = hashlib.sha256()
    for f in m_files.group(1).split(" + "):
        with open(os.path.join(ROOT, "paper_1004_4414_amd", "csrc", f.strip()), "rb") as fh:
            h.update(fh.read())
    if m_files.group(2) != h.hexdigest():
        return None
    return int(m_bytes.group(1))


def copy_bandwidth(torch, mib=1024, reps=5):
    """GB/s (read + write) of an elementwise kernel over `mib` MiB, timed with
    events: what a plain streaming copy reaches on this device"""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def _oracle_sample(seconds_budget):
    """(sites, steps, seconds) of the FP64 oracle stepping the bounded sample
    (a 64^3 box at the workload's volume fraction and fluid parameters)"""
    from oracle.oracle import Oracle
    from paper_1004_4414_amd import workloads as W
    n = 64
    count = W.sphere_count((n, n, n), 0.15, 5.0)
    p = W.params(nx=n, ny=n, nz=n, rho_init=(0.35, 0.35), noise_amp=0.01, g_br=0.08, seed=1003, force_average=1)
    parts = W.make_particles(W.random_sphere_positions((n, n, n), count, 5.0, seed=1003), 5.0)
    orc = Oracle(p)
    orc.add_particles(parts)
    steps = 0
    t0 = time.perf_counter()
    while True:
        orc.step(1)
        steps += 1
        dt = time.perf_counter() - t0
        if dt > seconds_budget or steps >= 200:
            break
    return n ** 3, steps, dt


def _oracle_worker(args):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    return _oracle_sample(args)


def cpu_baseline(seconds_budget=12.0):
    """The FP64 oracle on the host on a bounded sample of the workload: a 64^3
    box with the same volume fraction (75 spheres of radius 5) and fluid
    parameters, stepped for about `seconds_budget` on one core, then as
    independent copies on every core this process may use (the oracle itself
    is single-threaded)."""
    import multiprocessing as mp
    sites, steps, dt = _oracle_sample(seconds_budget)
    one = sites * steps / dt / 1e6
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(ncores, 16))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_worker, [seconds_budget] * workers)
    wall = time.perf_counter() - t0
    total = sum(s * k for s, k, _ in res)
    allc = total / max(wall, max(d for _, _, d in res)) / 1e6
    return dict(value=round(allc, 3), unit="MLUPS", cores=workers, kind="oracle",
                single_core_mlups=round(one, 3), host_cpus=os.cpu_count(), affinity_cpus=ncores,
                sample=f"64^3 box, {W_count()} spheres of radius 5 (volume fraction 0.15), g=0.08; "
                       f"one copy per core for about {seconds_budget:.0f} s each ({workers} copies), "
                       f"and one copy alone ({steps} steps); the 256^3 workload itself takes about "
                       f"{sites * 64 / (one * 1e6):.0f} s per oracle step on one core")


def W_count():
    from paper_1004_4414_amd import workloads as W
    return W.sphere_count((64, 64, 64), 0.15, 5.0)


def serving_leg(seconds_hint=None):
    """A short served trace on the default line: 8 jobs (edges 32-64, radii
    4-6, fractions 0.05-0.15, 200-400 steps, BF16 storage) arriving over half
    a second, through the continuous-batching server; jobs/hour and p50/p99
    time-to-result."""
    import torch
    from paper_1004_4414_amd import serving as S, workloads as W
    rng = __import__("numpy").random.Generator(__import__("numpy").random.PCG64(1006))
    jobs = []
    t = 0.0
    for k in range(8):
        t += float(rng.exponential(0.06))
        edge = int(rng.choice([32, 48, 64]))
        job = W._job(rng, edge, float(rng.uniform(0.5, 0.7)), float(rng.uniform(0.05, 0.15)),
                     float(rng.uniform(4.0, 6.0)), float(rng.uniform(60.0, 120.0)),
                     int(rng.integers(20, 41)) * 10, 1006 * 1000 + k)
        jobs.append(S.Job(job["params"], job["particles"], job["steps"], arrival=t,
                          contact_angle=job["contact_angle"], name=f"job{k}"))
    free, _ = torch.cuda.mem_get_info()
    small = min(jobs, key=lambda j: (j.params["nx"], j.steps))
    srv = S.Server(int(0.5 * free), precision="bf16", steps_per_launch=10, keep_density=(small.name,))
    out = srv.run(jobs)
    res = S.summary(out)
    err = next((S.density_error(r, small) for r in out if r.name == small.name and r.observables is not None), None)
    return dict(jobs_per_hour=round(res["jobs_per_hour"], 1), p50_s=round(res["p50_s"], 4),
                p99_s=round(res["p99_s"], 4), jobs=res["jobs"], failed=res["failed"], launches=srv.launches,
                batch_rebuilds=srv.batch_rebuilds, dtype="bf16", error_vs_fp64=err,
                workload="8 jobs, edges 32-64, radii 4-6, fractions 0.05-0.15, 200-400 steps, BF16 storage "
                         "(FP32 arithmetic), arrivals over about half a second")


def bench_ensemble(args):
    """Batched ensemble: 64 boxes (edges 32-96, ratios 50:50-80:20, particle
    fractions 0.05-0.25, radii 4-6, contact angles 60-120 degrees), FP32,
    2000 steps each.  Every distinct box edge gets its sweep variant from the
    autotuner; the boxes are then run (a) one job at a time with lb_step and
    (b) all resident together, advanced by graph launches of a batch."""
    import torch
    from paper_1004_4414_amd import lbm, workloads as W
    steps = args.steps or 2000
    k = 20 if steps % 20 == 0 else 2
    jobs = W.ensemble(64, seed=1004, steps=steps)
    tuned = {}
    t_tune = time.perf_counter()
    for j in jobs:
        e = j["params"]["nx"]
        if e not in tuned:
            tuned[e] = lbm.autotune(j["params"], j["particles"], "fp32", trial_steps=10)
    t_tune = time.perf_counter() - t_tune
    print(f"# autotuned {sorted((e, v[0], v[1]) for e, v in tuned.items())} in {t_tune:.1f} s", file=sys.stderr,
          flush=True)

    def make(j):
        kern, tile, _ = tuned[j["params"]["nx"]]
        lat = lbm.Lattice(j["params"], precision="fp32", kernel=kern, tile=tile)
        parts = {kk: v.copy() for kk, v in j["particles"].items()}
        parts["color"][:] = lbm.contact_angle_to_color(j["contact_angle"])
        lat.add_particles(parts)
        return lat

    sites = sum(j["params"]["nx"] ** 3 for j in jobs)
    # (a) one job at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    failed_alone = []
    for i, j in enumerate(jobs):
        lat = make(j)
        lat.step(steps)
        try:
            lat.synchronize()
        except lbm.LBError:  # the job went unstable: it is counted as not completed
            failed_alone.append(i)
        lat.close()
    t_alone = time.perf_counter() - t0
    print(f"# one at a time: {t_alone:.2f} s", file=sys.stderr, flush=True)
    # (b) resident batch, one graph launch per k steps of all 64 boxes
    lats = [make(j) for j in jobs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = lbm.Batch(lats, steps_per_launch=k)
    t_capture = time.perf_counter() - t0
    batch.step(steps // k)
    failed = []
    for i, lat in enumerate(lats):
        try:
            lat.synchronize()
        except lbm.LBError:
            failed.append(i)
    t_batch = time.perf_counter() - t0
    print(f"# batched: {t_batch:.2f} s (capture {t_capture:.2f} s)", file=sys.stderr, flush=True)
    batch.close()
    done = len(jobs) - len(failed)
    jph = done / t_batch * 3600.0
    return {
        "metric": f"jobs/hour (batched ensemble of 64 boxes, {steps} steps each)",
        "value": round(jph, 1), "unit": "jobs/hour", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(t_batch / steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ensemble64: 64 periodic boxes, edges {32,48,64,96}, ratios 50:50-80:20, "
                               "fractions 0.05-0.25, radii 4-6, contact angles 60-120 deg, FP32",
                   "sites": sites, "spheres": int(sum(len(j["particles"]["radius"]) for j in jobs)),
                   "steps_per_launch": k, "autotuned": {str(e): [v[0], list(v[1])] for e, v in tuned.items()}},
        "one_at_a_time": {"jobs_per_hour": round((len(jobs) - len(failed_alone)) / t_alone * 3600.0, 1),
                          "seconds": round(t_alone, 3), "failed_jobs": failed_alone},
        "batched": {"seconds": round(t_batch, 3), "capture_seconds": round(t_capture, 3),
                    "mlups": round(sites * steps / t_batch / 1e6, 1), "failed_jobs": failed},
        "speedup": round(t_alone / t_batch, 3),
    }


def bench_serving(args):
    """Serving trace, compressed: Poisson arrivals (20 jobs/min, arrival times
    divided by 60) of boxes with edges 48-192, radii 4-8 at fractions
    0.05-0.3, contact angles 45-135 degrees, 2000-20000 steps scaled by 1/20.
    The continuous-batching server (BF16 storage, admission by footprint)
    against one-at-a-time FP32 stepping."""
    import torch
    from paper_1004_4414_amd import serving as S, workloads as W
    k = 10
    trace = W.serving_trace(40, seed=1005, rate_per_min=20.0, time_scale=60.0, step_scale=0.05, step_quantum=k)
    jobs = [S.Job(t["params"], t["particles"], t["steps"], arrival=t["arrival"], contact_angle=t["contact_angle"],
                  name=f"job{i}") for i, t in enumerate(trace)]
    free, total = torch.cuda.mem_get_info()
    budget = int(0.6 * free)
    small = min(jobs, key=lambda j: (j.params["nx"], j.steps))
    srv = S.Server(budget, precision="bf16", steps_per_launch=k, keep_density=(small.name,))
    out = srv.run(jobs)
    served = S.summary(out)
    err = next((S.density_error(r, small) for r in out if r.name == small.name and r.observables is not None), None)
    print(f"# served: {served}, batch rebuilds {srv.batch_rebuilds}", file=sys.stderr, flush=True)
    alone = S.summary(S.run_alone(jobs, precision="fp32"))
    print(f"# one at a time (FP32): {alone}", file=sys.stderr, flush=True)
    return {
        "metric": "jobs/hour and p50/p99 time-to-result (served trace, continuous batching)",
        "value": round(served["jobs_per_hour"], 1), "unit": "jobs/hour", "n_gpus": 1,
        "steps": int(sum(j.steps for j in jobs)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "serving trace: 40 jobs, Poisson 20/min (times / 60), edges 48-192, radii 4-8, "
                               "fractions 0.05-0.3, angles 45-135 deg, 2000-20000 steps x 1/20; BF16 storage",
                   "budget_bytes": budget, "steps_per_launch": k},
        "served_bf16": served, "one_at_a_time_fp32": alone,
        "error_vs_fp64": err, "launches": srv.launches, "batch_rebuilds": srv.batch_rebuilds,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 100 for bijel256, 2000 per box for ensemble64)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--workload", default="bijel256")
    ap.add_argument("--tile", default="0,0,0", help="fused-kernel tile TX,TY,TZ (0 = automatic)")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "fp16", "bf16"],
                    help="population storage (default: the workload's); fp16/bf16 store deviations and compute in FP32")
    ap.add_argument("--develop", type=int, default=2000,
                    help="untimed steps before the warmup, so that the timed window is a developed state "
                         "(interfaces formed, spheres moving and in contact)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the short served trace of the default line")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the run, negate a buffer of this many MiB into another three times "
                         "(a kernel of known traffic that calibrates rocprofv3's FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: a lattice runs on one GPU "
              f"and independent boxes shard trivially, one or more per GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1004_4414_amd import lbm, workloads as W

    if args.copy_mib > 0:
        # one elementwise kernel per call that reads and writes copy_mib MiB
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        print(f"# calibration kernel: 3 launches, each {args.copy_mib} MiB read + {args.copy_mib} MiB written",
              file=sys.stderr, flush=True)

    if args.workload == "ensemble64":
        print(json.dumps(bench_ensemble(args)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    if args.steps is None:
        args.steps = 100

    p, parts, _, precision = W.config(args.workload)
    if args.precision:
        precision = args.precision
    N = p["nx"] * p["ny"] * p["nz"]
    tile = tuple(int(v) for v in args.tile.split(","))
    lat = lbm.Lattice(p, precision=precision, kernel=args.kernel, tile=tile)
    lat.add_particles(parts)
    print(f"# workload {args.workload}: {p['nx']}x{p['ny']}x{p['nz']}, {len(parts['radius'])} spheres, "
          f"{precision}, kernel {args.kernel}", file=sys.stderr, flush=True)
    if args.develop > 0:
        lat.step(args.develop)
        lat.synchronize()
        print(f"# developed for {args.develop} untimed steps", file=sys.stderr, flush=True)
    lat.step(args.warmup)
    lat.synchronize()
    lat.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat.synchronize()  # reports deferred device errors
    k_ms, k_n = lat.kernel_timing(0)
    s_ms, s_n = lat.kernel_timing(2)
    lat.enable_timing(False)
    obs = lat.observables()
    print(f"# {args.steps} steps in {elapsed:.3f} s; sweep {k_ms / max(k_n, 1):.3f} ms x {k_n}; "
          f"step (events) {s_ms / max(s_n, 1):.3f} ms; links {obs['n_links']}", file=sys.stderr, flush=True)

    mlups = N * args.steps / elapsed / 1e6
    fluid_sites = int((lat.owner() == -1).sum())
    copy_gbs = copy_bandwidth(torch)
    bps = algorithmic_bytes_per_site(precision)
    kern_name = {"auto": "twopass"}.get(args.kernel, args.kernel)
    traffic = measured_traffic(kern_name, precision, args.tile) if args.workload == "bijel256" else None
    sweep_s = k_ms / 1e3 / max(k_n, 1)
    achieved = bps * N / sweep_s / 1e9
    step_gbs = mlups * bps / 1e3
    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16", "bf16": "bf16"}[precision],
        "data": "synthetic",
        "config": {
            "workload": "bijel256: 256^3 periodic, 50:50 at 0.35+-0.01, g=0.08, tau=1, "
                        f"4806 spheres r=5 (volume fraction 0.15), neutral wettability, sphere fluid force averaged "
                        f"over two steps, {precision.upper()} populations"
            if args.workload == "bijel256" else args.workload,
            "sites": N,
            "spheres": len(parts["radius"]),
            "kernel": kern_name,
            "tile": args.tile,
            "storage": precision,
            "developed_steps_before_timing": args.develop,
        },
        # the dominant kernel: the sweep that collides and streams every
        # population (algorithmic bytes per site x sites / its mean launch time)
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": {"twopass": "k_collide_stream (second sweep of the two-pass step)",
                       "fused": "k_fused_step (the whole fluid step in one sweep)"}.get(kern_name, kern_name),
            "bytes_per_site": bps,
            "ms_per_launch": round(sweep_s * 1e3, 4),
            "copy_reference_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        # the whole step against the roofline: MLUPS x algorithmic bytes per
        # site over the peak, i.e. MLUPS as a fraction of the roofline MLUPS
        "step_roofline": {
            "achieved_gbs": round(step_gbs, 1),
            "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4),
            "roofline_mlups": round(HBM_PEAK_GBS * 1e3 / bps, 1),
            "frac_of_copy": round(step_gbs / copy_gbs, 4),
        },
        "mflups_fluid": round(mlups * fluid_sites / N, 1),
    }
    if not args.no_serving and args.workload == "bijel256":
        try:
            sv = serving_leg()
            line["jobs_per_hour"] = sv["jobs_per_hour"]
            line["p50_s"] = sv["p50_s"]
            line["p99_s"] = sv["p99_s"]
            line["serving"] = sv
        except Exception as e:  # reported, not hidden
            line["serving"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
