"""Trains the far-field closure's network on exact fields from this library.

    python -m paper_2203_11043_amd.closure_train --out DIR

Training data are snapshots of exact runs (the O(N^2) path, closure off):
Gaussian clouds of the single-cloud and batched-event workloads (holes
log-uniform in [2e3, 3e5], width 0.5 um (N/1000)^(1/3), shallow and deep
starting depths), recorded every 16 steps from the start through collection
or for at most 400 steps (fewer for the largest clouds, whose steps cost
most).  For every snapshot the library gives the exact Eq. (6) field,
the closure's exact near part, the grid charge and the grid placement; the
network's target at a carrier is the exact field minus the near part, in
units of K / h^2.  The loss is the relative squared error of the network's
output, interpolated to the carriers with the same Catmull-Rom weights as
the library.  Training seeds are 1000 and up, validation seeds 2000 and up.
The last part of training rounds weights and stored activations to bf16 as
the GPU does (straight-through gradients).

Writes DIR/closure_weights.npy (GCCD_CLOSURE_WEIGHTS float32 in the header's
order) and DIR/closure_train.json (data, settings, validation errors).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch
import torch.nn as nn
import torch.nn.functional as F

from . import gccd
from . import workloads as W

NG = 32
# (name, c_in, c_out, kernel) in the order of the weight array
LAYERS = [("e0a", 1, 16, 3), ("e0b", 16, 16, 3), ("e1a", 16, 32, 3), ("e1b", 32, 32, 3),
          ("e2a", 32, 32, 3), ("e2b", 32, 32, 3), ("b3a", 32, 32, 3), ("b3b", 32, 32, 3),
          ("d2", 64, 32, 3), ("d1", 64, 32, 3), ("d0", 48, 16, 3), ("head", 16, 3, 1)]

# CODATA 2018: K = q / (4 pi eps0 eps_r) in V um^2 / cm
_Q, _EPS0 = 1.602176634e-19, 8.8541878128e-12


def coulomb_K(eps_r: float) -> float:
    return _Q / (4.0 * math.pi * _EPS0 * eps_r) * 1e12 * 1e-2


def to_bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to bf16 (nearest even) in the forward pass, identity gradient."""
    return t + (t.to(torch.bfloat16).to(t.dtype) - t).detach()


class UNet(nn.Module):
    """The closure network: linear (no activation, no bias), so the far
    field it predicts scales with the charge and superposes."""

    def __init__(self):
        super().__init__()
        self.conv = nn.ModuleDict({n: nn.Conv3d(ci, co, k, padding=k // 2, bias=False)
                                   for n, ci, co, k in LAYERS})
        self.quant = False

    def _q(self, t):
        return to_bf16(t) if self.quant else t

    def _c(self, name, t, last=False):
        m = self.conv[name]
        w = self._q(m.weight)
        out = F.conv3d(t, w, padding=m.padding)
        return out if last else self._q(out)

    @staticmethod
    def _up(t):
        return F.interpolate(t, scale_factor=2, mode="trilinear", align_corners=False)

    def forward(self, rho):
        q = self._q
        x0 = q(rho)
        s0 = self._c("e0b", self._c("e0a", x0))
        s1 = self._c("e1b", self._c("e1a", q(F.avg_pool3d(s0, 2))))
        s2 = self._c("e2b", self._c("e2a", q(F.avg_pool3d(s1, 2))))
        b = self._c("b3b", self._c("b3a", q(F.avg_pool3d(s2, 2))))
        d2 = self._c("d2", torch.cat([q(self._up(b)), s2], 1))
        d1 = self._c("d1", torch.cat([q(self._up(d2)), s1], 1))
        d0 = self._c("d0", torch.cat([q(self._up(d1)), s0], 1))
        return self._c("head", d0, last=True)

    def flat_weights(self) -> np.ndarray:
        return np.concatenate([self.conv[n].weight.detach().float().cpu().numpy().ravel()
                               for n, *_ in LAYERS]).astype(np.float32)


def catmull_rom_sample(Fg: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Fg [B, 3, NG, NG, NG] (z, y, x), u [B, P, 3] node coordinates (x, y,
    z) -> [B, P, 3], cubic convolution over the 4 nodes per axis."""
    B, P = u.shape[0], u.shape[1]
    i = torch.clamp(torch.floor(u), 1, NG - 3)
    f = u - i
    i = i.long()
    f2, f3 = f * f, f * f * f
    w = torch.stack([0.5 * (-f3 + 2 * f2 - f), 0.5 * (3 * f3 - 5 * f2 + 2),
                     0.5 * (-3 * f3 + 4 * f2 + f), 0.5 * (f3 - f2)], dim=-1)  # [B,P,3,4]
    flat = Fg.reshape(B, 3, -1)
    out = torch.zeros(B, P, 3, device=Fg.device, dtype=Fg.dtype)
    for a in range(4):
        for b in range(4):
            for c in range(4):
                idx = ((i[..., 2] + a - 1) * NG + (i[..., 1] + b - 1)) * NG + (i[..., 0] + c - 1)
                vals = torch.gather(flat, 2, idx[:, None, :].expand(B, 3, P))  # [B,3,P]
                wt = w[..., 2, a] * w[..., 1, b] * w[..., 0, c]                  # [B,P]
                out = out + (vals * wt[:, None, :]).transpose(1, 2)
    return out


def snapshot(ctx, n, K, rng, points):
    """(rho [NG^3] / N, u [P,3], target [P,3] / N) of the current state."""
    E = gccd.gccd_field(ctx, n)
    near, _, rho, grid = gccd.gccd_closure_parts(ctx, n)
    pos, _ = gccd.gccd_positions(ctx, n)
    g = grid.cpu().numpy()
    h = float(g[3])
    pick = torch.as_tensor(rng.choice(n, min(points, n), replace=False), device=pos.device)
    u = (pos[:, pick].T - torch.as_tensor(g[:3], device=pos.device)) / h
    tgt = (E[:, pick] - near[:, pick]).T * (h * h / K)
    return (rho.reshape(1, NG, NG, NG) / n).float(), u.float(), (tgt / n).float()


def trajectory(seed, n, depth, steps, every, K, points, dev):
    """Snapshots of one exact run of a Gaussian cloud."""
    rng = np.random.default_rng(seed)
    x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, depth), seed, stream=9)
    d = dict(W.DEVICE, event=seed)
    ctx = gccd.gccd_init(gccd.Params.from_device(d))
    out = []
    try:
        t = [torch.as_tensor(v, dtype=torch.float64, device=dev) for v in (x, y, z)]
        gccd.gccd_load(ctx, *t)
        done = 0
        while True:
            out.append(snapshot(ctx, n, K, rng, points))
            if done >= steps:
                break
            k, na = gccd.gccd_run(ctx, W.DT_PS, every)
            done += every
            if na == 0:
                break
    finally:
        gccd.gccd_destroy(ctx)
    return out


def make_set(seeds, K, points, dev, log, steps=400, every=16, n_max=3e5):
    data = []
    for s in seeds:
        rng = np.random.default_rng(s)
        n = int(round(math.exp(rng.uniform(math.log(2e3), math.log(n_max)))))
        depth = float(rng.uniform(5.0, 60.0) if rng.random() < 0.6 else rng.uniform(60.0, 650.0))
        # at most about 4e12 pair interactions (about a second) per trajectory
        budget = max(every, min(steps, int(4e12 / (float(n) * n)) // every * every))
        t0 = time.time()
        snaps = trajectory(s, n, depth, budget, every, K, points, dev)
        data += snaps
        if s % 25 == 0 or time.time() - t0 > 2.0:
            log(f"seed {s}: n={n} depth={depth:.0f} um, {len(snaps)} snapshots "
                f"({time.time() - t0:.1f} s)")
    return data


def augment(rho, u, tgt, gen):
    """A random axis permutation and reflections (the Coulomb field is
    isotropic): grid axes (z, y, x) of rho, coordinate and field components."""
    perm = torch.randperm(3, generator=gen).tolist()       # new axis d <- old axis perm[d]
    flip = (torch.rand(3, generator=gen) < 0.5).tolist()
    # rho dims 1, 2, 3 are z, y, x = coordinate axes 2, 1, 0
    dims = [1 + (2 - perm[2 - a]) for a in range(3)]
    rho = rho.permute(0, *dims)
    u = u[:, perm]
    tgt = tgt[:, perm]
    for d in range(3):
        if flip[d]:
            rho = torch.flip(rho, dims=[1 + (2 - d)])
            u[:, d] = (NG - 1) - u[:, d]
            tgt[:, d] = -tgt[:, d]
    return rho, u, tgt


def rel_err(model, data, batch=8):
    """Mean over snapshots of ||pred - target|| / ||target||."""
    errs = []
    with torch.no_grad():
        for k in range(0, len(data), batch):
            part = data[k:k + batch]
            P = min(d[1].shape[0] for d in part)
            rho = torch.stack([d[0] for d in part])
            u = torch.stack([d[1][:P] for d in part])
            tgt = torch.stack([d[2][:P] for d in part])
            pred = catmull_rom_sample(model(rho), u)
            num = ((pred - tgt) ** 2).sum(dim=(1, 2))
            den = (tgt ** 2).sum(dim=(1, 2))
            errs += torch.sqrt(num / den).tolist()
    return float(np.mean(errs)), float(np.max(errs))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--train", type=int, default=1000, help="training trajectories (seeds 1000+)")
    ap.add_argument("--val", type=int, default=16, help="validation trajectories (seeds 2000+)")
    ap.add_argument("--points", type=int, default=2048)
    ap.add_argument("--iters", type=int, default=6000)
    ap.add_argument("--qat", type=float, default=0.2, help="final fraction trained with bf16")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    t_start = time.time()

    def log(msg):
        print(f"[{time.time() - t_start:7.1f} s] {msg}", flush=True)

    torch.backends.cudnn.enabled = False   # plain convolutions, no per-shape kernel tuning
    dev = torch.device("cuda", torch.cuda.current_device())
    K = coulomb_K(W.DEVICE["eps_r"])
    train = make_set(range(1000, 1000 + args.train), K, args.points, dev, log)
    val = make_set(range(2000, 2000 + args.val), K, args.points, dev, log)
    log(f"{len(train)} training and {len(val)} validation snapshots")

    torch.manual_seed(0)
    model = UNet().to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=args.lr)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=args.lr, total_steps=args.iters,
                                                pct_start=0.1, final_div_factor=200.0)
    gen = torch.Generator().manual_seed(0)
    q_from = int(args.iters * (1.0 - args.qat))
    for it in range(args.iters):
        model.quant = it >= q_from
        pick = torch.randint(len(train), (args.batch,), generator=gen).tolist()
        rho, u, tgt = [], [], []
        for k in pick:
            r, uu, tt = augment(train[k][0], train[k][1].clone(), train[k][2].clone(), gen)
            rho.append(r)
            u.append(uu)
            tgt.append(tt)
        P = min(v.shape[0] for v in u)
        rho = torch.stack(rho)
        u = torch.stack([v[:P] for v in u])
        tgt = torch.stack([v[:P] for v in tgt])
        pred = catmull_rom_sample(model(rho), u)
        loss = (((pred - tgt) ** 2).sum(dim=(1, 2)) / (tgt ** 2).sum(dim=(1, 2))).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        sched.step()
        if it % 100 == 0 or it == args.iters - 1:
            log(f"iter {it}: loss {loss.item():.3e}" + (" (bf16)" if model.quant else ""))
        if it % 500 == 0 or it == args.iters - 1:
            log(f"  validation relative error: mean {rel_err(model, val)[0]:.4f}")

    model.quant = True
    tr = rel_err(model, train)
    va = rel_err(model, val)
    log(f"final (bf16) relative far-field error: train {tr[0]:.4f}, validation {va[0]:.4f} "
        f"(max {va[1]:.4f})")
    w = model.flat_weights()
    assert w.size == gccd.CLOSURE_WEIGHTS
    np.save(os.path.join(args.out, "closure_weights.npy"), w)
    meta = dict(train_seeds=[1000, 1000 + args.train - 1], val_seeds=[2000, 2000 + args.val - 1],
                train_snapshots=len(train), val_snapshots=len(val), points=args.points,
                iters=args.iters, qat_fraction=args.qat, batch=args.batch, lr=args.lr,
                train_rel_err=tr[0], val_rel_err=va[0], val_rel_err_max=va[1],
                seconds=time.time() - t_start)
    with open(os.path.join(args.out, "closure_train.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {args.out}/closure_weights.npy")


if __name__ == "__main__":
    main()
