"""FP64 CPU oracle for the warm-start network (test infrastructure only).

The paper closes its introduction by pointing at hybrids of the PDE with
learned models but defines no network.  The warm start checked here is a
plain stack of six 3x3 convolutions (7 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3),
ReLU after the first five, zero "same" padding, fed with the hazy image, the
transmission and the broadcast atmospheric light, and trained by mean squared
error against converged solutions of the PDE with Adam.  Everything here is
float64 numpy, written tap by tap, so a reader can check each line against
the textbook definitions of cross-correlation, its two gradients, the ReLU,
the MSE loss and the Adam update (Kingma and Ba, 2015).

Nothing in the product package may import this module.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((7, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3))
# The network predicts u / OUT_SCALE; the warm start is OUT_SCALE times its output.
OUT_SCALE = 8.0


def param_count() -> int:
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unflatten(vec):
    """Flat parameter vector (per layer W[co][ci][3][3] then b[co]) -> [(W, b), ...]."""
    vec = np.asarray(vec, dtype=np.float64)
    out, off = [], 0
    for ci, co in LAYERS:
        W = vec[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = vec[off:off + co]
        off += co
        out.append((W, b))
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params])


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64.

    bfloat16 keeps the top 16 bits of a float32, so rounding a float32 to it is
    integer rounding of the low 16 bits.  Inputs are first rounded to float32.
    """
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def features(I: np.ndarray, t: np.ndarray, A) -> np.ndarray:
    """Network input: [I^R, I^G, I^B, t, A^R, A^G, A^B] as (7, H, W) float64."""
    I = np.asarray(I, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    H, W = t.shape
    Ab = np.broadcast_to(A[:, None, None], (3, H, W))
    return np.concatenate([I, t[None], Ab], axis=0)


def conv3x3(x: np.ndarray, Wt: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Cross-correlation with a 3x3 kernel, zero padding 1, stride 1.

    x (N, Ci, H, W), Wt (Co, Ci, 3, 3), b (Co,) ->
    y[n, o, j, i] = b[o] + sum_{c, dy, dx} Wt[o, c, dy, dx] x[n, c, j+dy-1, i+dx-1].
    """
    N, Ci, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    y = np.broadcast_to(np.asarray(b, dtype=np.float64)[None, :, None, None],
                        (N, Wt.shape[0], H, W)).copy()
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,nchw->nohw", Wt[:, :, dy, dx], xp[:, :, dy:dy + H, dx:dx + W])
    return y


def conv3x3_backward(x: np.ndarray, Wt: np.ndarray, g: np.ndarray):
    """Gradients of conv3x3 given dL/dy = g: returns (dL/dx, dL/dWt, dL/db)."""
    N, Ci, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dW = np.zeros_like(Wt, dtype=np.float64)
    dxp = np.zeros_like(xp, dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            dW[:, :, dy, dx] = np.einsum("nohw,nchw->oc", g, xp[:, :, dy:dy + H, dx:dx + W])
            dxp[:, :, dy:dy + H, dx:dx + W] += np.einsum("oc,nohw->nchw", Wt[:, :, dy, dx], g)
    db = g.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:H + 1, 1:W + 1], dW, db


def forward(x: np.ndarray, weights, act_round=None):
    """Run the six layers.  Returns (output, cache).

    ``act_round``, if given, is applied to the input and to every hidden
    activation after the ReLU (e.g. ``round_bf16`` to mirror bfloat16 storage);
    the last layer's output is not rounded.
    """
    rnd = act_round if act_round is not None else (lambda a: a)
    h = rnd(np.asarray(x, dtype=np.float64))
    cache = []
    n = len(weights)
    for k, (Wt, b) in enumerate(weights):
        z = conv3x3(h, Wt, b)
        cache.append((h, z))
        h = z if k == n - 1 else rnd(np.maximum(z, 0.0))
    return h, cache


def backward(cache, weights, gy: np.ndarray):
    """Back-propagate dL/d(output) through the stack; returns [(dW, db), ...]."""
    grads = [None] * len(weights)
    g = gy
    for k in range(len(weights) - 1, -1, -1):
        h, z = cache[k]
        if k != len(weights) - 1:
            g = g * (z > 0.0)
        dx, dW, db = conv3x3_backward(h, weights[k][0], g)
        grads[k] = (dW, db)
        g = dx
    return grads


def mse(y: np.ndarray, target: np.ndarray):
    """Mean squared error over every element and its gradient."""
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(param, grad, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns (param, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def warm_start(I, t, A, params, bf16: bool = True):
    """Starting iterate OUT_SCALE * net(features) for one image, (3, H, W).

    With bf16 the input, the weights and every hidden activation are rounded
    to bfloat16 as the GPU stores them (biases and the output stay wide).
    """
    x = features(I, t, A)[None]
    if bf16:
        params = [(round_bf16(W), b) for W, b in params]
        y, _ = forward(x, params, act_round=round_bf16)
    else:
        y, _ = forward(x, params)
    return OUT_SCALE * y[0]
