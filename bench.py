"""Benchmark of the charge-transport hot path on one MI355X.

One bench step = one simulation time step of a single 1e5-hole Gaussian
cloud (Eq. (6) all-pairs field + drift, mobility, diffusion, FP64 update and
collection, Sec. III.B).  The timed steps run as the library is used: one
gccd_run call (the host reads the counts every 32 steps), then the pixel
image of the collected holes (Sec. V.A).  Inputs are seeded synthetic
positions already resident in HBM.

Prints one JSON line: pair-interactions/s (the headline), carrier-steps/s,
the fraction of the FP32 vector peak, a roofline record for the Eq. (6)
kernel timed with HIP events on the library's stream, the FP64 CPU oracle
timed on a bounded sample of the same workload on the host cores, and the
far-field closure against the exact path on a 1e6-hole cloud.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3       # MI355X published FP32 vector peak
FLOP_PER_PAIR = 20             # N-body convention for one softened interaction
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "field_tiles_cloud_n100000_traffic.json")


def measured_traffic(n: int, tpt: int, chunks: int):
    """HBM bytes per Eq. (6) launch from the FETCH_SIZE / WRITE_SIZE counter
    runs recorded under profiles/, scaled by the copy-kernel calibration;
    None when the kernel source or the launch shape differs from the one the
    counters were taken on."""
    import hashlib
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, rec["kernel_source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if (sha != rec.get("kernel_source_sha256") or n != rec.get("n_holes", 100000)
            or tpt != rec.get("targets_per_thread") or chunks != rec.get("source_chunks")):
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline_batch(events, dev_dict, dt_ps, n_sample: int = 32, seed: int = 5) -> dict:
    """The oracle on a bounded sample of the batch: one time step of each of
    n_sample events drawn at random (each event alone, as the physics has it)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(events), size=min(n_sample, len(events)), replace=False)
    pairs = 0
    t0 = time.perf_counter()
    for e in pick:
        x, y, z = events[e]
        dev = oracle.Device(**dict(dev_dict))
        dev.event = int(dev_dict["event"]) + int(e)
        st = oracle.State(dev, x, y, z)
        na = st.n_active
        st.run(dt_ps, 1)
        pairs += na * len(x)
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one time step of {len(pick)} randomly drawn events of the batch, FP64, "
                      f"{dt:.1f} s wall"}


def cpu_baseline(w, max_seconds: float = 12.0) -> dict:
    """The oracle as it is, on the host cores: whole time steps of the same
    cloud (all n targets x n sources each) until about max_seconds."""
    import oracle
    dev = oracle.Device(**dict(w.device))
    st = oracle.State(dev, w.x, w.y, w.z)
    pairs = 0
    steps = 0
    t0 = time.perf_counter()
    while True:
        na = st.n_active
        st.run(w.dt_ps, 1)
        pairs += na * w.n
        steps += 1
        if time.perf_counter() - t0 > max_seconds or steps >= 8:
            break
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full time step(s) of the {w.n}-hole cloud on the host, "
                      f"FP64, {dt:.1f} s wall"}


def closure_leg(gccd, workloads, torch, n: int = 1000000, seed: int = 2000,
                closure_steps: int = 10, exact_steps: int = 3) -> dict:
    """The closure against the exact path on one large cloud (width
    0.5 um (n/1000)^(1/3), 300 um deep): time per step of each, measured the
    same way (one gccd_run call for the timed steps, after a warm-up call),
    from the same positions.  The accuracy figures come from the committed evaluation of
    whole runs (closure_eval.py), not from this short run."""
    import numpy as np
    from paper_2203_11043_amd import closure_eval
    if not os.path.exists(closure_eval.WEIGHTS):
        return None
    weights = closure_eval.load_weights()
    x, y, z = workloads.gaussian_cloud(n, workloads.cloud_sigma(n), (480.0, 480.0, 300.0), seed,
                                       stream=2)
    xs = [torch.as_tensor(v).cuda() for v in (x, y, z)]
    res = {}
    for name, use, warm, steps in (("closure", True, 5, closure_steps),
                                   ("exact", False, 2, exact_steps)):
        ctx = gccd.gccd_init(gccd.Params.from_device(dict(workloads.DEVICE, event=seed)))
        try:
            if use:
                gccd.gccd_set_closure(ctx, weights, 0)
            gccd.gccd_load(ctx, *xs)
            gccd.gccd_run(ctx, workloads.DT_PS, warm)
            torch.cuda.synchronize()
            s0 = gccd.gccd_stats(ctx)
            gccd.gccd_set_timing(ctx, True)
            t0 = time.perf_counter()
            gccd.gccd_run(ctx, workloads.DT_PS, steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s1 = gccd.gccd_stats(ctx)
        finally:
            gccd.gccd_destroy(ctx)
        cs = s1["carrier_steps"] - s0["carrier_steps"]
        pairs = s1["pair_interactions"] - s0["pair_interactions"]
        res[name] = {"ms_per_step": dt / steps * 1e3,
                     "field_ms_per_step": (s1["field_ms"] - s0["field_ms"]) / steps,
                     "carrier_steps_per_s": cs / dt,
                     "pair_interactions_per_s_equivalent": pairs / dt,
                     "closure_steps": s1["closure_steps"] - s0["closure_steps"],
                     "steps": steps, "warmup": warm}
    out = {"workload": f"single Gaussian cloud, n={n}, sigma={workloads.cloud_sigma(n):.2f} um, "
                       f"depth 300 um, seed {seed}",
           "closure": res["closure"], "exact": res["exact"],
           "speedup": res["exact"]["ms_per_step"] / res["closure"]["ms_per_step"]}
    ev = os.path.join(os.path.dirname(closure_eval.WEIGHTS), "closure_eval.json")
    if os.path.exists(ev):
        with open(ev) as f:
            rec = json.load(f)["results"]
        out["whole_run_accuracy"] = {
            "source": os.path.relpath(ev, ROOT),
            "var_x_rel": [r["var_x_rel"] for r in rec], "var_y_rel": [r["var_y_rel"] for r in rec],
            "image_l1_over_n": [r["image_l1_over_n"] for r in rec],
            "speedup_whole_run": [r["speedup"] for r in rec]}
    return out


DRIFT_BYTES_PER_CARRIER_STEP = 52   # x, y, z read and written (48), collection step read (4); a single event's carriers need no event read


def drift_leg(gccd, workloads, torch, n: int, steps: int, warm: int, cpu: bool) -> dict:
    """The paper's O(N) case (Sec. IV, Coulomb off): n holes drift and
    diffuse (Eqs. (1)-(4)), one step_update launch per time step.  A wide
    cloud 400 um deep, so that no hole is collected in the timed steps.  The
    oracle leg times whole Coulomb-off steps of the first 1e6 of the holes."""
    import numpy as np
    x, y, z = workloads.gaussian_cloud(n, 20.0, (480.0, 480.0, 400.0), 1, stream=30)
    d = dict(workloads.DEVICE, coulomb=0)
    xs = [torch.as_tensor(v).cuda() for v in (x, y, z)]
    ctx = gccd.gccd_init(gccd.Params.from_device(d))
    try:
        gccd.gccd_load(ctx, *xs)
        gccd.gccd_run(ctx, workloads.DT_PS, warm)
        torch.cuda.synchronize()
        s0 = gccd.gccd_stats(ctx)
        t0 = time.perf_counter()
        done, na = gccd.gccd_run(ctx, workloads.DT_PS, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = gccd.gccd_stats(ctx)
    finally:
        gccd.gccd_destroy(ctx)
    cs = s1["carrier_steps"] - s0["carrier_steps"]
    rate = cs / dt
    out = {"n": n, "steps": done, "travelling": na, "ms_per_step": dt / max(done, 1) * 1e3,
           "carrier_steps_per_s": rate,
           "roofline": {"bound": "hbm", "achieved": rate * DRIFT_BYTES_PER_CARRIER_STEP / 1e9,
                        "peak": 8000.0, "unit": "GB/s",
                        "frac": rate * DRIFT_BYTES_PER_CARRIER_STEP / 8e12,
                        "bytes_per_carrier_step": DRIFT_BYTES_PER_CARRIER_STEP}}
    if cpu:
        import oracle
        m = min(n, 1000000)
        st = oracle.State(oracle.Device(**d), x[:m], y[:m], z[:m])
        t0 = time.perf_counter()
        st.run(workloads.DT_PS, 2)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 2 * m / t, "unit": "carrier-steps/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"two Coulomb-off steps of {m} holes, FP64, {t:.1f} s"}
    return out


def sweep(gccd, workloads, torch, cpu: bool) -> dict:
    """The paper's timing protocol (Sec. IV, Fig. 4): 10 time steps of one
    cloud at each N, Coulomb on and off, on the GPU (median of 3 after one
    warm-up step) and, for the CPU baseline leg, the FP64 oracle on the host
    cores (once; Coulomb on up to N = 3e4, about 40 s in all).  Then whole
    runs to collection of the 1000-hole cloud, a 1e4-hole cloud and the
    muon track."""
    import numpy as np
    rows = []
    for n in (100, 300, 1000, 3000, 10000, 30000, 100000, 300000):
        w = workloads.single_cloud(n, seed=1, depth_um=300.0)
        row = {"n": n}
        for coulomb in (1, 0):
            d = dict(w.device, coulomb=coulomb)
            xs = [torch.as_tensor(v).cuda() for v in (w.x, w.y, w.z)]
            times = []
            for _ in range(3):
                ctx = gccd.gccd_init(gccd.Params.from_device(d))
                try:
                    gccd.gccd_load(ctx, *xs)
                    gccd.gccd_run(ctx, w.dt_ps, 1)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    gccd.gccd_run(ctx, w.dt_ps, 10)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                finally:
                    gccd.gccd_destroy(ctx)
            key = "on" if coulomb else "off"
            row[f"gpu_ms_10_steps_coulomb_{key}"] = float(np.median(times)) * 1e3
            if cpu and (coulomb == 0 or n <= 30000):
                import oracle
                st = oracle.State(oracle.Device(**d), w.x, w.y, w.z)
                t0 = time.perf_counter()
                st.run(w.dt_ps, 10)
                row[f"cpu_ms_10_steps_coulomb_{key}"] = (time.perf_counter() - t0) * 1e3
                row[f"speedup_coulomb_{key}"] = (row[f"cpu_ms_10_steps_coulomb_{key}"] /
                                                 row[f"gpu_ms_10_steps_coulomb_{key}"])
        rows.append(row)
    runs = []
    for name, w in (("cloud n=1000, depth 300 um", workloads.x_ray_cloud(seed=1)),
                    ("cloud n=10000", workloads.single_cloud(10000, seed=1)),
                    ("muon track n=62354", workloads.muon_track(seed=1))):
        xs = [torch.as_tensor(v).cuda() for v in (w.x, w.y, w.z)]
        ctx = gccd.gccd_init(gccd.Params.from_device(w.device))
        try:
            gccd.gccd_load(ctx, *xs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done, na = gccd.gccd_run(ctx, w.dt_ps, 20000)
            counts, nout = gccd.gccd_image(ctx, 0.0, 0.0, w.pitch_um, w.nx, w.ny)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = gccd.gccd_stats(ctx)
        finally:
            gccd.gccd_destroy(ctx)
        runs.append({"workload": name, "steps": done, "travelling_at_end": na,
                     "seconds": dt, "ms_per_step": dt / max(done, 1) * 1e3,
                     "pair_interactions": st["pair_interactions"],
                     "pair_interactions_per_s": st["pair_interactions"] / dt,
                     "collected_in_grid": int(counts.sum().item()),
                     "outside_grid": int(nout.item())})
    return {"cpu_cores": (__import__("oracle").num_threads() if cpu else None),
            "ten_steps": rows, "full_runs": runs}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 20; 200 for the drift workload, whose "
                         "steps are short enough that 20 end before the clock is up)")
    ap.add_argument("--workload", choices=("cloud", "batch", "closure", "sweep", "drift"),
                    default="cloud",
                    help="cloud: one 1e5-hole cloud (default); batch: 4096 clouds of "
                         "200-20000 holes in one launch; closure: only the closure-versus-"
                         "exact leg on the 1e6-hole cloud (--steps closure steps); sweep: the "
                         "paper's 10-step timing over N, Coulomb on and off, and whole runs; "
                         "drift: the Coulomb-off O(N) step on --n holes (2^24 by default)")
    ap.add_argument("--n", type=int, default=0, help="holes (0: 1e5, or 2^24 for drift)")
    ap.add_argument("--events", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tpt", type=int, default=0, help="targets per thread (0 = auto)")
    ap.add_argument("--chunks", type=int, default=0, help="source chunks (0 = auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--call-per-step", action="store_true",
                    help="one gccd_run call and one image per time step (a host round trip "
                         "per step) instead of one call for all timed steps")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch workload: keep the automatic launch shape instead of "
                         "measuring the candidates first (gccd_autotune)")
    ap.add_argument("--autotune", action="store_true",
                    help="single cloud: measure the candidate launch shapes first "
                         "(gccd_autotune) instead of the automatic shape")
    ap.add_argument("--no-closure", action="store_true",
                    help="skip the closure-versus-exact leg on the 1e6-hole cloud")
    ap.add_argument("--schedule", choices=("grid", "queue", "graph"), default="grid",
                    help="how gccd_run issues the steps (gccd_set_schedule)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (counter scale)")
    args = ap.parse_args()
    if args.warmup is None:
        args.warmup = 200 if args.workload == "drift" else 20

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not "
              "supported (the multi-GPU sharding is a design note, not code)", file=sys.stderr)
        return 2

    import torch
    from paper_2203_11043_amd import gccd, workloads

    torch.cuda.set_device(0)
    # a copy of known size first: its counters scale those of the kernels
    if args.copy_calibration_mib:
        a = torch.empty(args.copy_calibration_mib * (1 << 20) // 4, dtype=torch.float32,
                        device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    import numpy as np
    if args.workload == "sweep":
        res = sweep(gccd, workloads, torch, cpu=not args.no_cpu_baseline)
        big = res["ten_steps"][-1]
        print(json.dumps({
            "metric": "time of 10 simulation steps against N (Coulomb on and off), 1 GPU",
            "value": big["gpu_ms_10_steps_coulomb_on"], "unit": "ms per 10 steps at N=3e5",
            "n_gpus": 1, "steps": 10, "warmup": 1, "ms_per_step": big["gpu_ms_10_steps_coulomb_on"] / 10,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": {"workload": "single Gaussian clouds of 1e2-3e5 holes "
                                                        "300 um deep; whole runs of the 1000-hole "
                                                        "cloud, a 1e4 cloud and the muon track"},
            "sweep": res}), flush=True)
        return 0
    if args.workload == "drift":
        res = drift_leg(gccd, workloads, torch, args.n or (1 << 24), args.steps, args.warmup,
                        cpu=not args.no_cpu_baseline)
        print(json.dumps({
            "metric": "carrier-steps/s of the Coulomb-off step at 1 GPU",
            "value": res["carrier_steps_per_s"], "unit": "carrier-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"{res['n']} holes, Gaussian of 20 um at depth 400 um, "
                                   "Coulomb off (drift, mobility, diffusion, update)"},
            "roofline": res["roofline"], "cpu_baseline": res.get("cpu_baseline"),
            "drift": res}), flush=True)
        return 0
    if args.workload == "closure":
        res = closure_leg(gccd, workloads, torch, closure_steps=args.steps, exact_steps=2)
        if res is None:
            print("bench.py: no trained closure weights in the package", file=sys.stderr)
            return 1
        c = res["closure"]
        print(json.dumps({
            "metric": "carrier-steps/s of the far-field closure at 1 GPU (exact vs closure)",
            "value": c["carrier_steps_per_s"], "unit": "carrier-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": c["warmup"], "ms_per_step": c["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 pairs, bf16 network", "data": "synthetic",
            "config": {"workload": res["workload"]}, "closure": res}), flush=True)
        return 0
    if args.workload == "batch":
        events = workloads.batch_of_clouds(args.events, seed=args.seed)
        sizes = [len(e[0]) for e in events]
        offsets = np.concatenate([[0], np.cumsum(sizes)]).tolist()
        w = workloads.Workload(f"batch_{args.events}", *(np.concatenate([e[k] for e in events])
                                                        for k in range(3)))
    else:
        w = workloads.single_cloud(args.n or 100000, seed=args.seed)

    params = gccd.Params.from_device(w.device)
    ctx = gccd.gccd_init(params)
    gccd.gccd_set_launch(ctx, args.tpt, args.chunks)
    gccd.gccd_set_schedule(ctx, args.schedule)
    xs = [torch.as_tensor(v).cuda() for v in (w.x, w.y, w.z)]
    tuned = None
    if args.workload == "batch":
        gccd.gccd_load_events(ctx, offsets, *xs)

        def image():
            gccd.gccd_image_events(ctx, args.events, 0.0, 0.0, w.pitch_um, w.nx, w.ny)
    else:
        gccd.gccd_load(ctx, *xs)
        counts = torch.empty((w.ny, w.nx), dtype=torch.uint32, device="cuda")
        nout = torch.empty(1, dtype=torch.uint64, device="cuda")

        def image():
            gccd.gccd_image(ctx, 0.0, 0.0, w.pitch_um, w.nx, w.ny, counts, nout)
    # the batch is autotuned by default; the single cloud keeps the automatic
    # shape (the counters of the committed traffic record were taken in it,
    # and the tuner finds nothing faster there)
    want_tune = args.autotune if args.workload == "cloud" else not args.no_autotune
    if want_tune and not (args.tpt or args.chunks):
        tuned = gccd.gccd_autotune(ctx)

    def run(k):
        """k time steps, as the library is used: one gccd_run call (counts
        polled every 32 steps), then the image of the collected holes; with
        --call-per-step, one call and one image per step."""
        if args.call_per_step:
            done = 0
            for _ in range(k):
                done += gccd.gccd_run(ctx, w.dt_ps, 1)[0]
                image()
            return done
        done = gccd.gccd_run(ctx, w.dt_ps, k)[0]
        image()
        return done

    run(args.warmup)
    torch.cuda.synchronize()
    s0 = gccd.gccd_stats(ctx)
    gccd.gccd_set_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = gccd.gccd_stats(ctx)
    # The timed steps above record HIP events around every field launch,
    # which makes gccd_run issue them one by one.  The same number of steps
    # again without the events shows what the graph schedule gives.
    graph_pass = None
    if args.schedule == "graph":
        gccd.gccd_set_timing(ctx, False)
        torch.cuda.synchronize()
        g0 = gccd.gccd_stats(ctx)
        t2 = time.perf_counter()
        gdone = run(args.steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g1 = gccd.gccd_stats(ctx)
        graph_pass = {"steps": gdone, "ms_per_step": (t3 - t2) / max(gdone, 1) * 1e3,
                      "pair_interactions_per_s":
                          (g1["pair_interactions"] - g0["pair_interactions"]) / (t3 - t2),
                      "graph_replays": g1["graph_replays"] - g0["graph_replays"],
                      "graph_usable": g1["graph_usable"]}
    gccd.gccd_destroy(ctx)
    if done != args.steps:
        print(f"bench.py: only {done} of {args.steps} steps had travelling holes", file=sys.stderr)
        return 1

    elapsed = t1 - t0
    pairs = s1["pair_interactions"] - s0["pair_interactions"]
    csteps = s1["carrier_steps"] - s0["carrier_steps"]
    launches = s1["field_launches"] - s0["field_launches"]
    kern_s = (s1["field_ms"] - s0["field_ms"]) * 1e-3
    pair_rate = pairs / elapsed
    kern_tflops = FLOP_PER_PAIR * (pairs / launches) / (kern_s / launches) / 1e12

    out = {
        "metric": "pair-interactions/s & carrier-steps/s (exact vs closure) at 1 GPU, % FP32 peak",
        "value": pair_rate,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"single Gaussian hole cloud, exact all-pairs path: n={w.n}, "
                         f"sigma={workloads.cloud_sigma(w.n):.3f} um, depth {w.z.mean():.1f} um; "
                         "675 um CCD at 140 K, dt 10 ps, 64x64 image of 15 um pixels")
            if args.workload == "cloud" else
            (f"{args.events} independent Gaussian clouds in one launch, exact all-pairs path: "
             f"holes log-uniform in [200, 20000] (total {w.n}), sigma 0.5 um x (n/1000)^(1/3), "
             "depth uniform over 675 um; 140 K, dt 10 ps, one 64x64 image of 15 um pixels per "
             "event"),
            "n_holes": w.n,
            "n_events": s1["n_events"],
            "time_steps_per_step": 1,
            "calls": ("one gccd_run and one image per step" if args.call_per_step else
                      "one gccd_run for all timed steps (counts polled every 32 steps), "
                      "then the image"),
            "positions": "f64",
            "pair_arithmetic": ("f32, origin per workgroup; far tiles in the expanded-square form, "
                                "pairs closer than rho/4 with double-single differences, pairs "
                                "within 64 softening lengths in f64"
                                if s1["targets_per_thread"] == 1 else
                                "f32, origin per workgroup; pairs closer than rho/4 with "
                                "double-single differences, pairs within 64 softening lengths "
                                "in f64"),
            "targets_per_thread": s1["targets_per_thread"],
            "source_chunks": s1["source_chunks"],
            "max_source_chunks": s1["max_source_chunks"],
            "schedule": (args.schedule + ": the timed steps are issued one by one (per-launch "
                         "HIP events), see graph_pass for the replayed graphs"
                         if args.schedule == "graph" else args.schedule),
            "graph_pass": graph_pass,
            "tile_sources": s1["tile_sources"],
            "launch_shape": ("autotuned: targets per thread %d, source chunks %s, tile %d "
                             "sources (%.3f ms)" % (tuned[0], tuned[1] or "automatic",
                                                    s1["tile_sources"], tuned[2]))
                            if tuned else ("fixed" if (args.tpt or args.chunks) else "automatic"),
        },
        "carrier_steps_per_s": csteps / elapsed,
        "pct_fp32_peak": 100.0 * FLOP_PER_PAIR * pair_rate / (PEAK_FP32_TFLOPS * 1e12),
        "roofline": {
            "bound": "alu",
            "kernel": ("field_tiles_expanded (Eq. (6))" if s1["targets_per_thread"] == 1
                       else "field_tiles<%d> (Eq. (6))" % s1["targets_per_thread"]),
            "achieved": kern_tflops,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": kern_tflops / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(w.n, s1["targets_per_thread"], s1["source_chunks"]),
            "traffic_unit": "bytes per launch (HBM, counter-measured)",
            "avg_launch_ms": kern_s / launches * 1e3,
            "pairs_per_launch": pairs / launches,
            "flop_per_pair": FLOP_PER_PAIR,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = (cpu_baseline(w) if args.workload == "cloud" else
                               cpu_baseline_batch(events, w.device, w.dt_ps))
    if args.workload == "cloud" and not args.no_closure:
        out["closure"] = closure_leg(gccd, workloads, torch)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
