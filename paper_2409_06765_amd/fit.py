"""A synthetic fit from scratch: python -m paper_2409_06765_amd.fit [adc|mcmc|none] [steps]

Targets are renders of the seeded 100k-Gaussian SH-degree-3 scene from 16
views (400x400, focal 550, on a radius-4 sphere); the fit starts from 20,000
Gaussians with uniform random centres in [-1,1]^3, isotropic scale 0.02,
opacity 0.1 and a random base colour, and runs the training loop of
``train.GaussianTrainer`` with one view per step.  Prints the L1 loss and
Gaussian count every 500 steps and a JSON line with the time per step and
the final PSNR over the 16 views.
"""
import json
import sys
import time

import numpy as np
import torch

from . import scenes
from .train import GaussianTrainer, TrainConfig


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    strategy = argv[0] if argv else "adc"
    steps = int(argv[1]) if len(argv) > 1 else 3000
    sc = scenes.scene_uniform100k_sh3_800()
    g = np.random.default_rng(0)
    eyes = [4.0 * v / np.linalg.norm(v) for v in g.standard_normal((16, 3))]
    W = H = 400
    cams = scenes.cameras([scenes.look_at(e) for e in eyes], [scenes.intrinsics(550.0, W, H)] * 16, W, H)
    raw_gt = dict(means=sc["means"], quats=sc["quats"], log_scales=np.log(sc["scales"]),
                  logits=np.log(sc["opacities"] / (1 - sc["opacities"])), sh=sc["sh"])
    gt = GaussianTrainer(raw_gt, cams, torch.zeros((16, H, W, 3)), TrainConfig(strategy="none"), sh_degree=3)
    targets = torch.stack([gt.render([v])[-1]["image"].reshape(H, W, 3) for v in range(16)])
    del gt
    n0 = 20_000
    start = dict(means=g.uniform(-1, 1, (n0, 3)).astype(np.float32),
                 quats=np.tile(np.array([1, 0, 0, 0], np.float32), (n0, 1)),
                 log_scales=np.full((n0, 3), np.log(0.02), np.float32),
                 logits=np.full(n0, np.log(0.1 / 0.9), np.float32),
                 sh=np.concatenate([g.uniform(0, 1, (n0, 1, 3)), np.zeros((n0, 15, 3))], 1).astype(np.float32))
    cfg = TrainConfig(strategy=strategy, refine_start=300, refine_every=100, refine_stop=2500, reset_every=1500,
                      lr_decay_steps=steps, capacity_factor=8.0)
    tr = GaussianTrainer(start, cams, targets, cfg, sh_degree=3)
    losses = []
    t0 = time.perf_counter()
    for t in range(steps):
        losses.append(tr.step())
        if (t + 1) % 500 == 0:
            torch.cuda.synchronize()
            print(f"step {t + 1}: L1 {float(losses[-1]):.5f} N {tr.N} {time.perf_counter() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    psnr = []
    for v in range(16):
        img = tr.render([v])[-1]["image"].reshape(H, W, 3)
        psnr.append(10 * np.log10(1.0 / float(((img - targets[v]) ** 2).mean())))
    print(json.dumps(dict(strategy=strategy, steps=steps, ms_per_step=round(1e3 * dt / steps, 3), n_start=n0,
                          n_end=tr.N, l1_first=round(float(losses[0]), 5), l1_last=round(float(losses[-1]), 5),
                          psnr_db=round(float(np.mean(psnr)), 2),
                          finite=bool(torch.isfinite(tr.raw["means"]).all()))), flush=True)


if __name__ == "__main__":
    main()
