"""Pins of the oracle's readings of the two refinements Table II ablates but
the paper does not define: the guided filter (He, Sun and Tang) on t, and the
multiscale dark channel.  With no definition in the paper to check against,
they are pinned to brute force, closed forms and library routines."""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import dehaze_ref as o

pytestmark = pytest.mark.parametrize("seed", [0, 1])


def _brute_box_mean(x, r):
    H, W = x.shape
    out = np.empty_like(x, dtype=np.float64)
    for y in range(H):
        for xx in range(W):
            w = x[max(0, y - r):y + r + 1, max(0, xx - r):xx + r + 1]
            out[y, xx] = w.sum() / w.size
    return out


def _brute_guided(G, q, r, eps):
    H, W = G.shape
    a = np.empty((H, W))
    b = np.empty((H, W))
    for y in range(H):
        for x in range(W):
            g = G[max(0, y - r):y + r + 1, max(0, x - r):x + r + 1].ravel()
            v = q[max(0, y - r):y + r + 1, max(0, x - r):x + r + 1].ravel()
            cov = np.mean(g * v) - g.mean() * v.mean()
            var = np.mean(g * g) - g.mean() ** 2
            a[y, x] = cov / (var + eps)
            b[y, x] = v.mean() - a[y, x] * g.mean()
    return _brute_box_mean(a, r) * G + _brute_box_mean(b, r)


def test_box_mean_brute_force(seed):
    x = np.random.default_rng(seed).normal(size=(9, 13))
    for r in (0, 1, 3, 20):
        assert np.allclose(o.box_mean(x, r), _brute_box_mean(x, r), rtol=0, atol=1e-13)


def test_guided_filter_brute_force(seed):
    rng = np.random.default_rng(seed)
    G = rng.uniform(0, 1, size=(8, 11))
    q = rng.uniform(0, 1, size=(8, 11))
    for r, eps in ((1, 1e-3), (2, 1e-2), (5, 1e-4)):
        assert np.allclose(o.guided_filter(G, q, r, eps), _brute_guided(G, q, r, eps), rtol=0, atol=1e-12)


def test_guided_filter_closed_forms(seed):
    rng = np.random.default_rng(seed)
    G = rng.uniform(0, 1, size=(16, 19))
    # a constant input passes through: a = 0, b = the constant
    assert np.allclose(o.guided_filter(G, np.full(G.shape, 0.37), 3, 1e-3), 0.37, atol=1e-14)
    # an input that is an affine function of the guide is reproduced with eps = 0
    q = 0.6 * G + 0.15
    assert np.allclose(o.guided_filter(G, q, 2, 0.0), q, atol=1e-12)
    # eps -> infinity: a -> 0, b -> mean(q), output -> mean of the window means
    q = rng.uniform(0, 1, size=G.shape)
    far = o.guided_filter(G, q, 2, 1e12)
    assert np.allclose(far, o.box_mean(o.box_mean(q, 2), 2), atol=1e-10)
    # transposing guide and input transposes the output
    assert np.allclose(o.guided_filter(G.T, q.T, 3, 1e-3), o.guided_filter(G, q, 3, 1e-3).T, atol=1e-14)


def test_multiscale_transmission_reduces_and_averages(seed):
    img = synth.hazy_image(37, 41, 100 + seed, beta_haze=(0.5, 2.0), occlusion=True)
    I = img["I"]
    base = o.prior(I)
    p3 = o.with_params(dark_scales=3)
    assert o.scale_patches(15, 3) == [15, 7, 3]
    td, t = o.multiscale_transmission(I, base["A"], p3)
    # each scale's t_d from a library minimum filter (edge mode 'nearest' equals
    # a window clipped to the image for a minimum)
    ref = []
    for side in (15, 7, 3):
        m = np.stack([ndimage.minimum_filter(I[c].astype(np.float64), size=side, mode="nearest")
                      for c in range(3)])
        ref.append(np.min(m / base["A"][:, None, None], axis=0))
    assert np.allclose(td, np.mean(ref, axis=0), rtol=0, atol=1e-15)
    assert np.allclose(t, np.clip(1 - 0.95 * td, 0, 1), atol=1e-15)
    # one scale is the plain transmission
    td1, _ = o.multiscale_transmission(I, base["A"], o.with_params(dark_scales=1))
    assert np.array_equal(td1, base["t_d"])
    # a finer patch never gives a smaller minimum: t_d grows with the scales
    assert np.all(td >= base["t_d"] - 1e-15)


def test_prior_with_refinements(seed):
    img = synth.hazy_image(30, 34, 200 + seed, beta_haze=(0.5, 2.0), occlusion=True)
    I = img["I"]
    p = o.with_params(guided_radius=3, guided_eps=1e-3, dark_scales=2)
    pr = o.prior(I, p)
    guide = ((I[0].astype(np.float64) + I[1]) + I[2]) / 3.0
    want = np.clip(_brute_guided(guide, pr["t_raw"].astype(np.float32).astype(np.float64), 3, 1e-3), 0, 1)
    assert np.allclose(pr["t"], want, atol=1e-12)
    assert np.allclose(pr["lam"], o.adaptive_weight(pr["t"], p), atol=0)
    assert np.allclose(pr["phi"], o.reconstruction(I, pr["t"], pr["A"], p.t0), atol=0)
    # the defaults are the printed formulation
    assert o.DEFAULT.guided_radius == 0 and o.DEFAULT.dark_scales == 1
