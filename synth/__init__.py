"""Seeded synthetic hazy-image generator.

The paper evaluates on a real-world hazy dataset that is not published
(Section IV-A), so every workload here is synthetic.  This module only draws
inputs: a clear scene J, a depth map d, a true transmission t = exp(-beta * d),
a true atmospheric light A and the hazy observation given by the scattering
model of Section II-A, I = J t + A (1 - t), plus a little sensor noise.  It
holds none of the dehazing method's arithmetic (no dark channel, no
transmission estimate, no reconstruction, no PDE), so both the CPU oracle and
the GPU path can draw their inputs from it without sharing any of the method.

All randomness comes from numpy's PCG64 ``default_rng(seed)``; the same seed
always yields the same arrays on any machine.

Recipe (one image of H rows and W columns):

* J: per colour channel, 8 isotropic Gaussian blobs (centre uniform over the
  image, width U(0.05, 0.3) * max(H, W) pixels, amplitude U(-1, 1)) plus a
  linear ramp U(-1, 1) * x + U(-1, 1) * y with x, y in [0, 1]; min-max
  normalised to [0, 1].
* d: the same smooth generator (one channel) scaled to [0, 3]; with
  ``occlusion=True`` 3 to 6 random axis-aligned rectangles or half-planes of
  constant depth U(0, 3) are pasted over it, giving sharp depth edges.
* t = exp(-beta_haze * d), A = (0.80, 0.85, 0.90) + U(-0.05, 0.05)^3.
* I = J t + A (1 - t) + N(0, 0.005^2), stored as float32 and NOT clipped;
  the 8-bit variant is round(clip(I, 0, 1) * 255).
"""
from __future__ import annotations

import numpy as np

A_BASE = (0.80, 0.85, 0.90)
NOISE_STD = 0.005

# Size classes of the uneven-size batches (rows, cols).
BATCH_SIZES = ((256, 256), (480, 640), (720, 1280), (1080, 1920), (1536, 2048))


def _smooth_field(rng: np.random.Generator, H: int, W: int, n_blobs: int = 8) -> np.ndarray:
    """Sum of separable Gaussian blobs plus a linear ramp, min-max scaled to [0, 1]."""
    xs = np.arange(W, dtype=np.float64)
    ys = np.arange(H, dtype=np.float64)
    f = np.zeros((H, W), dtype=np.float64)
    scale = float(max(H, W))
    for _ in range(n_blobs):
        cx = rng.uniform(0.0, 1.0) * W
        cy = rng.uniform(0.0, 1.0) * H
        width = rng.uniform(0.05, 0.3) * scale
        amp = rng.uniform(-1.0, 1.0)
        gx = np.exp(-((xs - cx) ** 2) / (2.0 * width * width))
        gy = np.exp(-((ys - cy) ** 2) / (2.0 * width * width))
        f += amp * np.outer(gy, gx)
    ax = rng.uniform(-1.0, 1.0)
    ay = rng.uniform(-1.0, 1.0)
    xn = xs / max(W - 1, 1)
    yn = ys / max(H - 1, 1)
    f += ax * xn[None, :] + ay * yn[:, None]
    lo, hi = f.min(), f.max()
    if hi - lo < 1e-300:
        return np.zeros_like(f)
    return (f - lo) / (hi - lo)


def _occlude(rng: np.random.Generator, d: np.ndarray) -> np.ndarray:
    """Paste 3-6 constant-depth rectangles or half-planes over a depth map."""
    H, W = d.shape
    d = d.copy()
    for _ in range(int(rng.integers(3, 7))):
        depth = rng.uniform(0.0, 3.0)
        if rng.uniform() < 0.5:
            y0, y1 = sorted(rng.integers(0, H + 1, size=2))
            x0, x1 = sorted(rng.integers(0, W + 1, size=2))
            d[y0:y1, x0:x1] = depth
        else:
            axis = int(rng.integers(0, 2))
            cut = int(rng.integers(0, (H if axis == 0 else W) + 1))
            upper = rng.uniform() < 0.5
            if axis == 0:
                if upper:
                    d[:cut, :] = depth
                else:
                    d[cut:, :] = depth
            else:
                if upper:
                    d[:, :cut] = depth
                else:
                    d[:, cut:] = depth
    return d


def hazy_image(H: int, W: int, seed: int, beta_haze=1.0, occlusion: bool = False) -> dict:
    """Draw one synthetic hazy RGB image.

    ``beta_haze`` is either a number or a (lo, hi) pair drawn uniformly.
    Returns a dict with planar (channel-first) arrays:
      J (3,H,W) f64, d (H,W) f64, t_true (H,W) f64, A_true (3,) f64,
      I (3,H,W) float32, I_u8 (3,H,W) uint8, beta_haze (float), seed (int).
    """
    if H < 1 or W < 1:
        raise ValueError("image must have at least one pixel")
    rng = np.random.default_rng(seed)
    if isinstance(beta_haze, (tuple, list)):
        beta = float(rng.uniform(beta_haze[0], beta_haze[1]))
    else:
        beta = float(beta_haze)
    J = np.stack([_smooth_field(rng, H, W) for _ in range(3)])
    d = 3.0 * _smooth_field(rng, H, W)
    if occlusion:
        d = _occlude(rng, d)
    t = np.exp(-beta * d)
    A = np.asarray(A_BASE, dtype=np.float64) + rng.uniform(-0.05, 0.05, size=3)
    noise = rng.normal(0.0, NOISE_STD, size=(3, H, W))
    I64 = J * t[None] + A[:, None, None] * (1.0 - t[None]) + noise
    I = I64.astype(np.float32)
    I_u8 = np.rint(np.clip(I64, 0.0, 1.0) * 255.0).astype(np.uint8)
    return {"J": J, "d": d, "t_true": t, "A_true": A, "I": I, "I_u8": I_u8,
            "beta_haze": beta, "seed": int(seed)}


def scattering_forward(J: np.ndarray, t: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Noise-free scattering model I = J t + A (1 - t) in float64 (planar J)."""
    A = np.asarray(A, dtype=np.float64)
    return J * t[None] + A[:, None, None] * (1.0 - t[None])


# ---------------------------------------------------------------- workloads
def small_image(seed: int = 1000):
    """64x64 single image, beta_haze = 1.0, smooth depth."""
    return hazy_image(64, 64, seed, beta_haze=1.0, occlusion=False)


def megapixel_image(seed: int = 2000):
    """1024x1024 single image, beta_haze ~ U(0.5, 2.0), depth with occlusion edges."""
    return hazy_image(1024, 1024, seed, beta_haze=(0.5, 2.0), occlusion=True)


def batch_sizes(n: int, seed: int) -> list:
    """Image sizes of an uneven batch, uniform over the five size classes."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(BATCH_SIZES), size=n)
    return [BATCH_SIZES[int(i)] for i in idx]


def _window_field(rng, ch: int, cw: int, ys: np.ndarray, xs: np.ndarray, n_blobs: int = 8):
    """The _smooth_field recipe on a virtual ch x cw canvas, evaluated at rows
    ys and columns xs (canvas coordinates); returns (values, canvas min, max)
    with the min and max taken on a stride-8 grid of the canvas plus the window."""
    scale = float(max(ch, cw))
    blobs = [(rng.uniform(0.0, 1.0) * cw, rng.uniform(0.0, 1.0) * ch, rng.uniform(0.05, 0.3) * scale,
              rng.uniform(-1.0, 1.0)) for _ in range(n_blobs)]
    ax, ay = rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0)

    def ev(yv, xv):
        f = np.zeros((yv.size, xv.size))
        for cx, cy, width, amp in blobs:
            f += amp * np.outer(np.exp(-((yv - cy) ** 2) / (2 * width * width)),
                                np.exp(-((xv - cx) ** 2) / (2 * width * width)))
        return f + ax * (xv / max(cw - 1, 1))[None, :] + ay * (yv / max(ch - 1, 1))[:, None]

    win = ev(ys, xs)
    coarse = ev(np.arange(0, ch, 8, dtype=np.float64), np.arange(0, cw, 8, dtype=np.float64))
    return win, min(win.min(), coarse.min()), max(win.max(), coarse.max())


def hazy_window(H: int, W: int, seed: int, canvas=(1080, 1920), beta_haze=(0.5, 2.5), occlusion: bool = True) -> dict:
    """An H x W window of a virtual canvas-sized scene drawn with the recipe
    of hazy_image (blob widths, ramps and occluders in canvas units), so a
    small image carries the object scales of a large one.  The window's
    offset is drawn uniformly; fields are min-max scaled with the canvas range
    (estimated on a stride-8 grid).  Same keys as hazy_image."""
    ch, cw = canvas
    if H > ch or W > cw:
        raise ValueError("window larger than the canvas")
    rng = np.random.default_rng(seed)
    beta = float(rng.uniform(*beta_haze)) if isinstance(beta_haze, (tuple, list)) else float(beta_haze)
    oy, ox = int(rng.integers(0, ch - H + 1)), int(rng.integers(0, cw - W + 1))
    ys = np.arange(oy, oy + H, dtype=np.float64)
    xs = np.arange(ox, ox + W, dtype=np.float64)
    J = []
    for _ in range(3):
        f, lo, hi = _window_field(rng, ch, cw, ys, xs)
        J.append(np.clip((f - lo) / max(hi - lo, 1e-300), 0.0, 1.0))
    J = np.stack(J)
    f, lo, hi = _window_field(rng, ch, cw, ys, xs)
    d = 3.0 * np.clip((f - lo) / max(hi - lo, 1e-300), 0.0, 1.0)
    if occlusion:
        for _ in range(int(rng.integers(3, 7))):
            depth = rng.uniform(0.0, 3.0)
            if rng.uniform() < 0.5:
                y0, y1 = sorted(rng.integers(0, ch + 1, size=2))
                x0, x1 = sorted(rng.integers(0, cw + 1, size=2))
                m = ((ys >= y0) & (ys < y1))[:, None] & ((xs >= x0) & (xs < x1))[None, :]
            else:
                axis = int(rng.integers(0, 2))
                cut = int(rng.integers(0, (ch if axis == 0 else cw) + 1))
                upper = rng.uniform() < 0.5
                v = ys if axis == 0 else xs
                side = (v < cut) if upper else (v >= cut)
                m = side[:, None] & np.ones((1, W), bool) if axis == 0 else np.ones((H, 1), bool) & side[None, :]
            d = np.where(m, depth, d)
    t = np.exp(-beta * d)
    A = np.asarray(A_BASE, dtype=np.float64) + rng.uniform(-0.05, 0.05, size=3)
    noise = rng.normal(0.0, NOISE_STD, size=(3, H, W))
    I64 = J * t[None] + A[:, None, None] * (1.0 - t[None]) + noise
    return {"J": J, "d": d, "t_true": t, "A_true": A, "I": I64.astype(np.float32),
            "I_u8": np.rint(np.clip(I64, 0.0, 1.0) * 255.0).astype(np.uint8), "beta_haze": beta, "seed": int(seed),
            "offset": (oy, ox)}


def uneven_batch(n: int = 64, base_seed: int = 3000, beta_haze=(0.5, 2.5), sizes=None):
    """Uneven-size batch; image k uses seed base_seed + k."""
    if sizes is None:
        sizes = batch_sizes(n, base_seed)
    return [hazy_image(h, w, base_seed + k, beta_haze=beta_haze, occlusion=True)
            for k, (h, w) in enumerate(sizes)]


# ---------------------------------------------------------------- network init
CNN_LAYERS = ((7, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3))


def cnn_init_params(seed: int = 0, gain: float = 1.0) -> np.ndarray:
    """He-normal initial weights, zero biases, as one float32 vector laid out
    per layer as W[co][ci][3][3] followed by b[co]."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CNN_LAYERS:
        std = gain * np.sqrt(2.0 / (ci * 9))
        parts.append(rng.normal(0.0, std, size=co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
