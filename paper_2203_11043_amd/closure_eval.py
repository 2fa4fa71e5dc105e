"""Compares the far-field closure with the exact path on the same GPU.

    python -m paper_2203_11043_amd.closure_eval --out DIR [--n 1000000] [--seeds 2000]

For every seed, a Gaussian cloud of n holes (width 0.5 um (n/1000)^(1/3),
5 um at 1e6, centred 300 um deep under the corner of four pixels) runs to
collection twice from the same positions and Philox stream: once on the
exact O(N^2) path and once with the closure.  Reported per seed: steps, time
per step, the variances and covariance of the collected positions, and the
64x64 images (15 um pixels): the sum of absolute pixel differences over N
and the largest pixel difference.  Writes DIR/closure_eval.json.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import gccd
from . import workloads as W

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closure",
                       "closure_weights.npy")


def load_weights(path: str = WEIGHTS) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    if w.size != gccd.CLOSURE_WEIGHTS:
        raise ValueError(f"{path}: {w.size} weights, expected {gccd.CLOSURE_WEIGHTS}")
    return w.astype(np.float32)


def run_to_collection(x, y, z, weights, event, log, chunk=64, max_steps=20000):
    d = dict(W.DEVICE, event=event)
    ctx = gccd.gccd_init(gccd.Params.from_device(d))
    try:
        if weights is not None:
            gccd.gccd_set_closure(ctx, weights, 0)
        dev = torch.device("cuda", torch.cuda.current_device())
        gccd.gccd_load(ctx, *[torch.as_tensor(v, dtype=torch.float64, device=dev)
                              for v in (x, y, z)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        while steps < max_steps:
            done, na = gccd.gccd_run(ctx, W.DT_PS, chunk)
            steps += done
            if na == 0 or done == 0:
                break
            if steps % (2 * chunk) == 0:
                log(f"    step {steps}: {na} travelling, "
                    f"{(time.perf_counter() - t0) / steps * 1e3:.2f} ms/step")
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        pos, cs = gccd.gccd_positions(ctx, len(x))
        counts, nout = gccd.gccd_image(ctx, 0.0, 0.0, W.PITCH_UM, 64, 64)
        st = gccd.gccd_stats(ctx)
        return dict(steps=steps, seconds=secs, n_active=int(na),
                    pos=pos.cpu().numpy(), image=counts.cpu().numpy().astype(np.int64),
                    n_outside=int(nout.item()), closure_steps=int(st["closure_steps"]),
                    carrier_steps=int(st["carrier_steps"]))
    finally:
        gccd.gccd_destroy(ctx)


def moments(pos):
    x, y = pos[0], pos[1]
    return float(np.var(x)), float(np.var(y)), float(np.cov(x, y)[0, 1])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=1000000)
    ap.add_argument("--depth", type=float, default=300.0)
    ap.add_argument("--seeds", type=int, nargs="+", default=[2000])
    ap.add_argument("--weights", default=WEIGHTS)
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    t_start = time.time()

    def log(msg):
        print(f"[{time.time() - t_start:7.1f} s] {msg}", flush=True)

    weights = load_weights(args.weights)
    results = []
    for seed in args.seeds:
        x, y, z = W.gaussian_cloud(args.n, W.cloud_sigma(args.n), (480.0, 480.0, args.depth),
                                   seed, stream=2)
        log(f"seed {seed}: n={args.n}, sigma={W.cloud_sigma(args.n):.3f} um, "
            f"depth {args.depth} um: closure run")
        clo = run_to_collection(x, y, z, weights, seed, log)
        log(f"  closure: {clo['steps']} steps, {clo['seconds'] / clo['steps'] * 1e3:.2f} ms/step")
        log("  exact run")
        ex = run_to_collection(x, y, z, None, seed, log)
        log(f"  exact: {ex['steps']} steps, {ex['seconds'] / ex['steps'] * 1e3:.2f} ms/step")
        me, mc = moments(ex["pos"]), moments(clo["pos"])
        diff = np.abs(ex["image"] - clo["image"])
        r = dict(seed=seed, n=args.n, depth_um=args.depth,
                 steps_exact=ex["steps"], steps_closure=clo["steps"],
                 closure_steps=clo["closure_steps"],
                 ms_per_step_exact=ex["seconds"] / ex["steps"] * 1e3,
                 ms_per_step_closure=clo["seconds"] / clo["steps"] * 1e3,
                 speedup=(ex["seconds"] / ex["steps"]) / (clo["seconds"] / clo["steps"]),
                 var_x_exact=me[0], var_y_exact=me[1], cov_xy_exact=me[2],
                 var_x_closure=mc[0], var_y_closure=mc[1], cov_xy_closure=mc[2],
                 var_x_rel=mc[0] / me[0] - 1.0, var_y_rel=mc[1] / me[1] - 1.0,
                 image_l1_over_n=float(diff.sum()) / args.n, image_max_abs=int(diff.max()),
                 image_peak=int(ex["image"].max()),
                 charge_exact=int(ex["image"].sum()) + ex["n_outside"] + ex["n_active"],
                 charge_closure=int(clo["image"].sum()) + clo["n_outside"] + clo["n_active"])
        log("  " + json.dumps({k: (round(v, 6) if isinstance(v, float) else v)
                               for k, v in r.items()}))
        results.append(r)
    with open(os.path.join(args.out, "closure_eval.json"), "w") as f:
        json.dump(dict(results=results, weights=os.path.relpath(args.weights)), f, indent=1)
    log(f"wrote {args.out}/closure_eval.json")


if __name__ == "__main__":
    main()
