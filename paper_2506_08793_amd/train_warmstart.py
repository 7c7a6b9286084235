"""Train the warm-start network on converged solutions of the plain method.

    python -m paper_2506_08793_amd.train_warmstart --n 2048 --size 256 --steps 6000 --out <path>
    python -m paper_2506_08793_amd.train_warmstart --n 256 --size 1080x1920 --canvas 0 --batch 2 \
        --chunk 32 --seed0 8000 --steps 6000 --out <path>      (the shipped default)

Images are seeded synthetic hazy images (seeds 4000 + k, beta_haze ~
U(0.5, 2.5), occlusion edges) of size x size pixels cut from virtual
1920 x 1080 scenes, so their object scales match the full-HD images the
network warm-starts (--canvas 0 draws whole size x size scenes instead).
Targets are u* - B: the lagged-diffusivity batch solve run cold to relative
residual 1e-5, minus the analytic start B = Phi / lambda, which the network
corrects.  Progress goes to stdout.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np
import torch

from . import binding as b
from . import warmstart as ws


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--size", default="256", help="side of square images, or HxW")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed0", type=int, default=4000)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--canvas", default="1080x1920", help="HxW of the virtual scene, or 0")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    import synth  # seeded input generator (repository root)

    ctx = b.Context(0)
    H, W = (int(v) for v in args.size.split("x")) if "x" in args.size else (int(args.size),) * 2
    t0 = time.time()
    imgs = []
    canvas = None if args.canvas in ("0", "") else tuple(int(v) for v in args.canvas.split("x"))
    for k in range(args.n):
        if canvas:
            imgs.append(synth.hazy_window(H, W, args.seed0 + k, canvas=canvas)["I"])
        else:
            imgs.append(synth.hazy_image(H, W, args.seed0 + k, beta_haze=(0.5, 2.5), occlusion=True)["I"])
        if (k + 1) % 64 == 0:
            print(f"generated {k + 1}/{args.n} ({time.time() - t0:.1f} s)", flush=True)
    print(f"generated {args.n} images {H}x{W} in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    data, stats = None, []
    parts = []
    for k in range(0, args.n, args.chunk):
        d, st = ws.solve_targets(ctx, imgs[k:k + args.chunk], chunk=args.chunk)
        parts.append(d)
        stats += st
        outs = [s["outer"] for s in st]
        print(f"solved {k + len(st)}/{args.n}: outer mean {np.mean(outs):.0f} max {max(outs)} "
              f"({time.time() - t0:.1f} s)", flush=True)
    data = tuple(torch.cat([p[i] for p in parts]) for i in range(4))
    conv = sum(s["converged"] for s in stats)
    print(f"targets: {conv}/{len(stats)} converged to 1e-5", flush=True)
    b.dehaze_cnn_set_weights(ctx, synth.cnn_init_params(args.init_seed))
    hist = ws.train(ctx, data, args.steps, batch=args.batch, lr=args.lr, log_every=500)
    meta = {"images": args.n, "size": [H, W], "canvas": args.canvas, "seeds": [args.seed0, args.seed0 + args.n - 1],
            "beta_haze": [0.5, 2.5], "steps": args.steps, "batch": args.batch, "lr": args.lr,
            "final_loss": hist[-1][1], "targets_converged": conv, "init_seed": args.init_seed,
            "target": "u* - Phi/lambda"}
    ws.save(ctx, args.out, meta)
    print(f"saved {args.out}: {meta}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
