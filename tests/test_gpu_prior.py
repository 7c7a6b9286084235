"""GPU front end vs the FP64 oracle: dark channel, 8-bit dark channel and A
bit-exact, t_d bit-exact against the float32 rounding of the oracle's
quotient, t / lambda / Phi within tolerances derived from float32 rounding."""
import numpy as np
import pytest

import synth
from gpu_util import ctx, dev, host, require_gpu, say
from oracle import dehaze_ref as o

pytestmark = pytest.mark.gpu

# (H, W, seed): single pixel, thin strips, ragged multi-tile shapes, the
# 64x64 workload, a patch larger than the image.
SHAPES = [(1, 1, 11), (3, 2, 12), (5, 300, 13), (300, 5, 14), (9, 13, 15), (37, 53, 16), (64, 64, 1000),
          (130, 70, 17), (257, 190, 18)]

# t = clamp(1 - omega t_d): float32 t_d (exact rounding) and a float64
# evaluation rounded once give |t - t_oracle| <= 2^-25 omega + 2^-25.
T_TOL = 2.0 ** -24
# lambda = lambda0 exp(-beta (1 - t)): relative error beta |dt| + 2^-24.
LAM_RTOL = 3.0 * T_TOL + 2.0 ** -23
# Phi = (I - A (1 - t)) / max(t, t0): |dPhi/dt| <= (|A| + |Phi|) / t0.
def _phi_tol(phi, t0=0.1):
    return T_TOL * (1.0 + np.abs(phi)) / t0 + 2.0 ** -23 * np.abs(phi) + 1e-12


def _run(H, W, seed, dtype, layout, A_in=None):
    require_gpu()
    import paper_2506_08793_amd as d
    img = synth.hazy_image(H, W, seed, beta_haze=(0.5, 2.0), occlusion=True)
    if dtype == "u8":
        arr = img["I_u8"]
        I32 = o.unit_from_u8(arr)
    else:
        arr = img["I"]
        I32 = arr
    ref = o.prior(I32, o.DEFAULT, A=A_in)
    I_t = dev(arr if layout == "CHW" else arr.transpose(1, 2, 0))
    outs = ("dark", "t_d", "t", "lam", "phi") + (("dark_u8",) if dtype == "u8" else ())
    say(f"prior H={H} W={W} seed={seed} {dtype} {layout} A_in={A_in is not None}")
    A_dev = dev(np.asarray(A_in, dtype=np.float32)) if A_in is not None else None
    out = d.dehaze_prior(ctx(), I_t, layout=layout, outputs=outs, A_in=A_dev)
    got = {k: host(v) for k, v in out.items() if not k.startswith("_")}
    return img, arr, ref, got


@pytest.mark.parametrize("H,W,seed", SHAPES)
@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("layout", ["CHW", "HWC"])
def test_prior_parity(H, W, seed, dtype, layout):
    img, arr, ref, got = _run(H, W, seed, dtype, layout)
    assert np.array_equal(got["dark"], ref["dc"].astype(np.float32))
    assert np.array_equal(got["A"].astype(np.float64), ref["A"])
    assert np.array_equal(got["t_d"].view(np.uint32), ref["t_d"].astype(np.float32).view(np.uint32))
    assert np.max(np.abs(got["t"] - ref["t"])) <= T_TOL
    assert np.max(np.abs(got["lam"] - ref["lam"]) / ref["lam"]) <= LAM_RTOL
    assert np.all(np.abs(got["phi"] - ref["phi"]) <= _phi_tol(ref["phi"]))
    if dtype == "u8":
        want = o.dark_channel(o.patch_min(arr.astype(np.float64), 15)).astype(np.uint8)
        assert np.array_equal(got["dark_u8"], want)


def test_prior_with_given_airlight():
    A = [0.82, 0.87, 0.93]
    img, arr, ref, got = _run(70, 90, 21, "f32", "CHW", A_in=A)
    assert np.array_equal(got["A"], np.asarray(A, dtype=np.float32))
    ref = o.prior(img["I"], o.DEFAULT, A=np.asarray(A, dtype=np.float32).astype(np.float64))
    assert np.array_equal(got["t_d"], ref["t_d"].astype(np.float32))
    assert np.all(np.abs(got["phi"] - ref["phi"]) <= _phi_tol(ref["phi"]))


def test_prior_airlight_ties_on_flat_codes():
    # many exactly equal dark-channel values: the tie rule decides A
    require_gpu()
    import paper_2506_08793_amd as d
    rng = np.random.default_rng(4)
    codes = rng.integers(200, 203, size=(3, 120, 97), dtype=np.uint8)
    I32 = o.unit_from_u8(codes)
    ref = o.prior(I32)
    say("prior ties 120x97")
    out = d.dehaze_prior(ctx(), dev(codes), outputs=("dark",))
    assert np.array_equal(host(out["A"]).astype(np.float64), ref["A"])
    assert np.array_equal(host(out["dark"]), ref["dc"].astype(np.float32))


def test_prior_full_megapixel_workload():
    img, arr, ref, got = _run(1024, 1024, 2000, "f32", "CHW")
    assert np.array_equal(got["dark"], ref["dc"].astype(np.float32))
    assert np.array_equal(got["A"].astype(np.float64), ref["A"])
    assert np.array_equal(got["t_d"], ref["t_d"].astype(np.float32))
    assert np.all(np.abs(got["phi"] - ref["phi"]) <= _phi_tol(ref["phi"]))


@pytest.mark.parametrize("patch", [1, 3, 31])
def test_prior_other_patch_sizes(patch):
    require_gpu()
    import paper_2506_08793_amd as d
    img = synth.hazy_image(45, 77, 30 + patch, beta_haze=1.0)
    p = d.dehaze_params_default(patch=patch)
    ref = o.prior(img["I"], o.with_params(patch=patch))
    say(f"prior patch={patch}")
    out = d.dehaze_prior(ctx(), dev(img["I"]), params=p, outputs=("dark", "t_d"))
    assert np.array_equal(host(out["dark"]), ref["dc"].astype(np.float32))
    assert np.array_equal(host(out["A"]).astype(np.float64), ref["A"])


def test_prior_rejects_bad_arguments():
    require_gpu()
    import paper_2506_08793_amd as d
    img = dev(synth.hazy_image(8, 8, 1)["I"])
    for kw in ({"patch": 4}, {"patch": 33}, {"t0": 0.0}, {"eps": -1.0}, {"omega": 1.5}, {"strip_rows": -1},
               {"lane_columns": 3}):
        with pytest.raises(d.DehazeError) as e:
            d.dehaze_prior(ctx(), img, params=d.dehaze_params_default(**kw))
        assert e.value.code == -1


# Refinements (readings of the guided filter and multiscale dark channel that
# Table II ablates).  t_d of several scales is a mean of per-scale float32
# t_d summed in float64: within one float32 ulp of the oracle's float64 mean.
# The guided filter is linear in its input with gain at most about
# max|g - mean g| / (var g + eps) per window (~30 at eps = 1e-3), so a one-ulp
# difference in its input moves the output by at most ~30 ulps; with equal
# inputs only the summation order differs (one rounding at the end).
@pytest.mark.parametrize("H,W,seed", [(37, 53, 16), (64, 64, 1000), (130, 70, 17), (5, 300, 13), (1, 1, 11)])
@pytest.mark.parametrize("radius,scales", [(0, 2), (0, 3), (4, 1), (8, 3), (20, 2)])
def test_prior_refinements_parity(H, W, seed, radius, scales):
    require_gpu()
    import paper_2506_08793_amd as d
    img = synth.hazy_image(H, W, seed, beta_haze=(0.5, 2.0), occlusion=True)
    q = o.with_params(guided_radius=radius, dark_scales=scales, guided_eps=1e-3)
    ref = o.prior(img["I"], q)
    say(f"prior refinements H={H} W={W} r={radius} scales={scales}")
    p = d.dehaze_params_default(guided_radius=radius, dark_scales=scales, guided_eps=1e-3)
    out = d.dehaze_prior(ctx(), dev(img["I"]), params=p, outputs=("dark", "t_d", "t", "lam", "phi"))
    got = {k: host(v) for k, v in out.items() if not k.startswith("_")}
    assert np.array_equal(got["dark"], ref["dc"].astype(np.float32))
    assert np.array_equal(got["A"].astype(np.float64), ref["A"])
    td32 = ref["t_d"].astype(np.float32)
    if scales == 1:
        assert np.array_equal(got["t_d"], td32)
    else:
        assert np.all(np.abs(got["t_d"] - td32) <= np.spacing(td32))
    if radius == 0:
        t_tol = T_TOL if scales == 1 else 2.0 * T_TOL
    else:
        t_tol = 2.0 ** -23 if scales == 1 else 30 * 2.0 ** -24
    err = np.max(np.abs(got["t"] - ref["t"]))
    say(f"  max |dt| {err:.3e} (bound {t_tol:.3e})")
    assert err <= t_tol
    # lambda and Phi of the library's own t
    t_own = got["t"].astype(np.float64)
    lam_own = o.adaptive_weight(t_own)
    phi_own = o.reconstruction(img["I"], t_own, got["A"].astype(np.float64), 0.1)
    assert np.max(np.abs(got["lam"] - lam_own) / lam_own) <= 2.0 ** -23
    assert np.all(np.abs(got["phi"] - phi_own) <= 2.0 ** -23 * np.abs(phi_own) + 1e-12)


def test_batch_front_end_applies_refinements():
    # the batch's own front end (t estimated inside) equals dehaze_prior +
    # dehaze_solve with the same parameters, bit for bit
    require_gpu()
    import paper_2506_08793_amd as d
    imgs = [synth.hazy_image(h, w, 40 + k, beta_haze=(0.5, 2.0), occlusion=True)["I"]
            for k, (h, w) in enumerate([(48, 40), (33, 70)])]
    p = d.dehaze_params_default(guided_radius=6, dark_scales=2, max_outer=20, rel_tol=0.0)
    say("batch front end with refinements")
    ub, _, tb, Ab = d.dehaze_batch(ctx(), [dev(I) for I in imgs], params=p, want_t=True)
    for k, I in enumerate(imgs):
        pr = d.dehaze_prior(ctx(), dev(I), params=p, outputs=("t",))
        assert np.array_equal(host(tb[k]), host(pr["t"]))
        us, _ = d.dehaze_solve(ctx(), dev(I), pr["t"], pr["A"], params=p)
        assert np.array_equal(host(ub[k]), host(us))
