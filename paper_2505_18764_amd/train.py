"""Fitting loop over the differentiable rasterizer: Adam on raw Gaussian parameters, one or more
views per step (several views render in the same launches and their gradients are summed on the
device), L2 photometric loss against target images.

Parameters are kept raw (means, log-scales, quaternions, opacity logits, SH) and activated in
torch (exp, sigmoid; the projection normalises quaternions), then rendered with
GaussianRasterizeFn; the rasterizer's forward state is rematerialised in its backward, so the
only per-view memory beyond the parameters is the framebuffer and the O(N) splat records.

Run as a module for the 500k-Gaussian, 8-camera, 1280x720 fitting workload:
    python -m paper_2505_18764_amd.train [--steps 300] [--n 500000] [--views-per-step 1]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from .render import RasterConfig, Workspace, rasterize_gaussians


class GaussianParams(torch.nn.Module):
    def __init__(self, means3d, scales, quats, opacities, sh, sh_degree=3):
        super().__init__()
        dev = means3d.device
        self.means = torch.nn.Parameter(means3d.clone())
        self.log_scales = torch.nn.Parameter(torch.log(scales.clamp_min(1e-8)).clone())
        self.quats = torch.nn.Parameter(quats.clone())
        o = opacities.clamp(1e-4, 1 - 1e-4)
        self.logits = torch.nn.Parameter(torch.log(o / (1 - o)).clone())
        self.sh = torch.nn.Parameter(sh.clone())
        self.sh_degree = sh_degree
        self.to(dev)

    def activated(self):
        return (self.means, torch.exp(self.log_scales), self.quats, torch.sigmoid(self.logits),
                self.sh)


def render(params: GaussianParams, cam, cfg: RasterConfig, ws: Workspace):
    return rasterize_gaussians(*params.activated(), cam, cfg, ws)


def fit(params: GaussianParams, cams, targets, steps: int, lr: float = 1e-3, cfg=None,
        log_every: int = 10, callback=None, views_per_step: int = 1):
    """Adam (torch defaults, lr) on all raw parameters. Step k renders views
    (k B + j) % len(cams), j < B = views_per_step, in one batched call (B > 1) and takes the mean
    squared error over them."""
    cfg = cfg or RasterConfig(sh_degree=params.sh_degree)
    ws = Workspace(params.means.device)
    opt = torch.optim.Adam(params.parameters(), lr=lr)
    hist = []
    B = views_per_step
    tgt = torch.stack(list(targets)) if B > 1 else None
    for k in range(steps):
        if B > 1:
            vs = [(k * B + j) % len(cams) for j in range(B)]
            img, _ = render(params, [cams[v] for v in vs], cfg, ws)
            loss = torch.mean((img - tgt[vs]) ** 2)
        else:
            v = k % len(cams)
            img, _ = render(params, cams[v], cfg, ws)
            loss = torch.mean((img - targets[v]) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if k % log_every == 0 or k == steps - 1:
            hist.append((k, float(loss.detach())))
            if callback:
                callback(k, hist[-1][1])
    return hist


def main():
    import synth
    ap = argparse.ArgumentParser()
    c = synth.CFG4
    ap.add_argument("--steps", type=int, default=c["steps"])
    ap.add_argument("--n", type=int, default=c["n_train"])
    ap.add_argument("--width", type=int, default=c["width"])
    ap.add_argument("--height", type=int, default=c["height"])
    ap.add_argument("--fb-format", default="f16")
    ap.add_argument("--views-per-step", type=int, default=1)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    fx = c["fx"] * args.width / c["width"]
    cams = [synth.camera_ring(k, c["cameras"], width=args.width, height=args.height, fx=fx)
            for k in range(c["cameras"])]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hidden = synth.scene3d(args.n, seed=c["seed_hidden"])
    train0 = synth.scene3d(args.n, seed=c["seed_train"])
    cfg = RasterConfig(fb_format=args.fb_format, reduce_mode="tile")
    ws = Workspace(dev)
    with torch.no_grad():
        targets = [rasterize_gaussians(t(hidden.means3d), t(hidden.scales), t(hidden.quats),
                                       t(hidden.opacities), t(hidden.sh), cam, cfg, ws)[0].clone()
                   for cam in cams]
    params = GaussianParams(t(train0.means3d), t(train0.scales), t(train0.quats),
                            t(train0.opacities), t(train0.sh))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = fit(params, cams, targets, args.steps, lr=c["lr"], cfg=cfg,
               callback=lambda k, l: print(f"step {k} loss {l:.6f}", flush=True),
               views_per_step=args.views_per_step)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"steps": args.steps, "n": args.n, "resolution": [args.width, args.height],
                      "views_per_step": args.views_per_step,
                      "s_per_step": dt / args.steps, "loss_first": hist[0][1],
                      "loss_last": hist[-1][1], "history": hist}))


if __name__ == "__main__":
    main()
