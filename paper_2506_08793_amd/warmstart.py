"""Training and storage of the warm-start network.

The warm start is B + net(I, t, A), where B = Phi / lambda is the analytic
start (warm_start = 2): the solution of lambda u = Phi, to which the main PDE
reduces where u is smooth.  The network learns the correction u* - B from the
hazy image, the transmission and the atmospheric light.  Its training targets
are produced by the plain method itself: the lagged-diffusivity batch solve
run cold (from Phi) to the relative residual 1e-5, minus B from the same
library (a zero-step solve from warm_start = 2).  Everything below drives the
C ABI: the solves, the forward/backward passes and the Adam steps run in the
library's kernels; torch holds device memory and forms u* - B.

Weights are stored as a little-endian float32 file (the parameter vector in
the library's layout) next to a JSON file with the training metadata.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import binding as b

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def solve_targets(ctx, images, params=None, chunk: int = 64):
    """Network targets u* - B for a list of planar float32 images.

    u* is the converged solution (cold start), B the analytic start of the
    same image.  images: list of numpy (3, H, W) arrays of one size.  Returns
    device tensors (I, t, A, u_star - B) stacked over images, plus per-image
    stats of the solves.
    """
    p = params or b.dehaze_params_default(max_outer=6000, rel_tol=1e-5)
    pb = b.dehaze_params_default(warm_start=2, max_outer=0, rel_tol=0.0)
    Is, ts, As, us, stats = [], [], [], [], []
    for k in range(0, len(images), chunk):
        dev = [torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in images[k:k + chunk]]
        u, st, t, A = b.dehaze_batch(ctx, dev, params=p, want_t=True)
        base, _, _, _ = b.dehaze_batch(ctx, dev, params=pb, t=t, A=A, stats=False)
        Is += dev
        us += [ui - bi for ui, bi in zip(u, base)]
        ts += t
        As += A
        stats += st
    return (torch.stack(Is), torch.stack(ts), torch.stack(As), torch.stack(us)), stats


def train(ctx, data, steps: int, batch: int = 16, lr: float = 2e-3, lr_final: float = 1e-4, seed: int = 0,
          log_every: int = 100, log=print):
    """Adam on random mini-batches of whole images; cosine decay lr -> lr_final."""
    I, t, A, u = data
    n, _, H, W = I.shape
    rng = np.random.default_rng(seed)
    ws = b.cnn_workspace(batch, H, W, True)
    hist = []
    t0 = time.time()
    for s in range(steps):
        idx = torch.from_numpy(rng.choice(n, size=batch, replace=False)).cuda()
        frac = s / max(1, steps - 1)
        lr_s = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
        want = (s % log_every == 0) or s == steps - 1
        loss = b.dehaze_cnn_train_step(ctx, I[idx].contiguous(), t[idx].contiguous(), A[idx].contiguous(),
                                       u[idx].contiguous(), lr_s, ws=ws, want_loss=want)
        if want:
            hist.append((s, loss))
            if log:
                log(f"step {s} loss {loss:.5e} lr {lr_s:.2e} ({time.time() - t0:.1f} s)")
    return hist


def save(ctx, path: str, meta: dict) -> None:
    w = b.dehaze_cnn_get_weights(ctx)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    w.astype("<f4").tofile(path)
    with open(path + ".json", "w") as f:
        json.dump({**meta, "param_count": int(w.size)}, f, indent=1)


def load(ctx, path: str) -> dict:
    w = np.fromfile(path, dtype="<f4")
    b.dehaze_cnn_set_weights(ctx, w)
    meta_path = path + ".json"
    if os.path.exists(meta_path):
        with open(meta_path) as f:
            return json.load(f)
    return {}


def default_weights_path() -> str:
    """The shipped network for full-HD warm starts: trained on 256 whole
    1920x1080 images (seeds 8000+).  weights_path(256) is the one trained on
    2048 windows of 256x256 (seeds 4000+)."""
    return weights_path(1080)


def weights_path(size: int) -> str:
    return os.path.join(WEIGHTS_DIR, f"warmstart_{size}.f32")
