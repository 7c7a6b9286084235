"""Pins of the oracle's front end (dark channel, A, t, lambda, Phi) against
brute force, library routines and closed forms of Sections II-A and II-D."""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi

import synth
from oracle import dehaze_ref as o


def test_u8_conversion_is_correctly_rounded():
    codes = np.arange(256, dtype=np.uint8)
    got = o.unit_from_u8(codes)
    # numpy's float32 division is IEEE correctly rounded
    want = codes.astype(np.float32) / np.float32(255.0)
    assert got.dtype == np.float32
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def _brute_patch_min(I, patch):
    C, H, W = I.shape
    r = patch // 2
    out = np.empty((C, H, W))
    for c in range(C):
        for j in range(H):
            for i in range(W):
                best = np.inf
                for jj in range(max(0, j - r), min(H, j + r + 1)):
                    for ii in range(max(0, i - r), min(W, i + r + 1)):
                        best = min(best, float(I[c, jj, ii]))
                out[c, j, i] = best
    return out


@pytest.mark.parametrize("H,W,patch", [(1, 1, 15), (3, 5, 3), (9, 4, 15), (17, 23, 5), (20, 16, 15)])
def test_patch_min_brute_force_and_scipy(H, W, patch):
    rng = np.random.default_rng(H * 100 + W)
    I = rng.uniform(-0.1, 1.1, size=(3, H, W)).astype(np.float32)
    got = o.patch_min(I, patch)
    assert np.array_equal(got, _brute_patch_min(I, patch))
    for c in range(3):
        lib = ndi.minimum_filter(I[c], size=patch, mode="nearest")
        assert np.array_equal(got[c].astype(np.float32), lib)


def test_patch_min_u8_codes_commute_with_conversion():
    rng = np.random.default_rng(7)
    codes = rng.integers(0, 256, size=(3, 31, 29), dtype=np.uint8)
    m_codes = o.patch_min(codes.astype(np.float64), 15)
    m_unit = o.patch_min(o.unit_from_u8(codes), 15)
    assert np.array_equal(o.unit_from_u8(m_codes.astype(np.uint8)).astype(np.float64), m_unit)


def test_patch_min_rejects_even_patch():
    with pytest.raises(ValueError):
        o.patch_min(np.zeros((3, 4, 4)), 4)


def _brute_airlight(I, dc, divisor):
    C, H, W = I.shape
    n = H * W
    k = max(1, n // divisor)
    keyed = sorted(range(n), key=lambda q: (-float(dc.reshape(-1)[q]), q))[:k]
    flat = I.reshape(3, -1).astype(np.float64)
    best = None
    for q in keyed:
        s = (flat[0, q] + flat[1, q]) + flat[2, q]
        if best is None or s > best[0] or (s == best[0] and q < best[1]):
            best = (s, q)
    return flat[:, best[1]], best[1]


@pytest.mark.parametrize("seed,H,W", [(0, 40, 60), (1, 50, 50), (2, 7, 300), (3, 1, 1)])
def test_airlight_brute_force_with_ties(seed, H, W):
    rng = np.random.default_rng(seed)
    # 8-bit codes give many exactly equal dark-channel values and sums
    codes = rng.integers(180, 256, size=(3, H, W), dtype=np.uint8)
    I = o.unit_from_u8(codes)
    dc = o.dark_channel(o.patch_min(I, 15))
    A, q = o.atmospheric_light(I, dc, 1000)
    A2, q2 = _brute_airlight(I, dc, 1000)
    assert q == q2 and np.array_equal(A, A2)


def test_airlight_finds_constructed_bright_region():
    # a haze-opaque region (t = 0) of known colour wins both the dark-channel
    # ranking and the brightness test
    H, W = 60, 80
    rng = np.random.default_rng(3)
    I = rng.uniform(0.0, 0.5, size=(3, H, W)).astype(np.float32)
    Atrue = np.array([0.81, 0.86, 0.91], dtype=np.float32)
    I[:, 10:40, 20:60] = Atrue[:, None, None]
    dc = o.dark_channel(o.patch_min(I, 15))
    A, q = o.atmospheric_light(I, dc, 1000)
    assert np.array_equal(A, Atrue.astype(np.float64))
    # lowest index among the tied pixels whose whole patch lies in the region
    assert q == (10 + 7) * W + (20 + 7)


def test_dcp_closed_form_transmission():
    # Section II-D: if some channel of J vanishes in every patch and t, A are
    # exact, the dark channel of I/A is 1 - t and the estimate is 1 - omega (1 - t).
    H, W = 48, 40
    rng = np.random.default_rng(11)
    J = rng.uniform(0.0, 1.0, size=(3, H, W))
    zero_ch = rng.integers(0, 3, size=(H // 8 + 1, W // 8 + 1))
    for jb in range(zero_ch.shape[0]):
        for ib in range(zero_ch.shape[1]):
            J[zero_ch[jb, ib], jb * 8:(jb + 1) * 8, ib * 8:(ib + 1) * 8] = 0.0
    t_true = 0.37
    A = np.array([0.8, 0.85, 0.9])
    I = synth.scattering_forward(J, np.full((H, W), t_true), A)
    m = o.patch_min(I, 15)
    td, t = o.transmission(m, A, 0.95)
    assert np.allclose(td, 1.0 - t_true, rtol=0, atol=1e-15)
    assert np.allclose(t, 1.0 - 0.95 * (1.0 - t_true), rtol=0, atol=1e-15)
    _, t1 = o.transmission(m, A, 1.0)
    assert np.allclose(t1, t_true, rtol=0, atol=1e-15)


def test_transmission_clamped_and_rejects_bad_airlight():
    m = np.stack([np.array([[1.2, -0.1]])] * 3)
    td, t = o.transmission(m, np.ones(3), 0.95)
    assert t.min() >= 0.0 and t.max() <= 1.0 and t[0, 1] == 1.0 and t[0, 0] == 0.0
    with pytest.raises(ValueError):
        o.transmission(m, np.array([0.5, 0.0, 0.5]), 0.95)


def test_adaptive_weight_closed_form():
    p = o.DEFAULT
    t = np.array([[0.0, 0.5, 1.0]])
    lam = o.adaptive_weight(t, p)
    assert lam[0, 2] == p.lambda0
    assert abs(lam[0, 0] - p.lambda0 * np.exp(-p.beta_lambda)) < 1e-16
    assert abs(lam[0, 1] - 0.5 * np.exp(-1.5)) < 1e-16
    assert np.all(np.diff(lam[0]) > 0)          # the printed formula rises with t
    assert np.all(o.adaptive_weight(t, o.with_params(adaptive=False)) == p.lambda0)


def test_reconstruction_round_trip():
    # Section II-A: Phi inverts the scattering model wherever t >= t0
    rng = np.random.default_rng(5)
    H, W = 33, 21
    J = rng.uniform(0.0, 1.0, size=(3, H, W))
    t = rng.uniform(0.1, 1.0, size=(H, W))
    A = np.array([0.77, 0.83, 0.94])
    I = synth.scattering_forward(J, t, A)
    phi = o.reconstruction(I, t, A, 0.1)
    assert np.max(np.abs(phi - J)) < 1e-13
    # below t0 the divisor is t0: Phi = J t / t0
    t_low = rng.uniform(0.0, 0.1, size=(H, W))
    I_low = synth.scattering_forward(J, t_low, A)
    phi_low = o.reconstruction(I_low, t_low, A, 0.1)
    assert np.max(np.abs(phi_low - J * t_low / 0.1)) < 1e-13


def test_prior_on_generated_image_is_consistent():
    img = synth.small_image()
    pr = o.prior(img["I"])
    assert pr["A"].shape == (3,)
    assert np.all(pr["A"] > 0)
    # A is the input colour at the chosen pixel
    q = pr["A_index"]
    assert np.array_equal(pr["A"], img["I"].reshape(3, -1)[:, q].astype(np.float64))
    assert pr["lam"].min() >= 0.5 * np.exp(-3.0) - 1e-15 and pr["lam"].max() <= 0.5
