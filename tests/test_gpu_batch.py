"""GPU batch path: uneven-size images solved together by the lagged-diffusivity
scheme with per-image stopping, checked against the FP64 oracle, against the
one-image entry points and against itself on graph replay."""
import numpy as np
import pytest

import synth
from gpu_util import ctx, dev, host, require_gpu, say
from oracle import dehaze_ref as o

pytestmark = pytest.mark.gpu

U_TOL = 1e-4
ACCURATE = dict(inner_rtol=1e-4, max_inner=200, inner_refine=3)
SIZES = [(24, 24), (40, 31), (17, 50), (1, 1), (65, 33)]


def _images(sizes, base_seed, dtype="f32"):
    imgs = [synth.hazy_image(h, w, base_seed + k, beta_haze=(0.5, 2.5), occlusion=True)
            for k, (h, w) in enumerate(sizes)]
    arrs = [im["I_u8"] if dtype == "u8" else im["I"] for im in imgs]
    I32 = [o.unit_from_u8(a) if dtype == "u8" else a for a in arrs]
    return arrs, I32


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_batch_fixed_steps_matches_oracle_and_single(dtype):
    require_gpu()
    import paper_2506_08793_amd as d
    arrs, I32 = _images(SIZES, 500, dtype)
    p = d.dehaze_params_default(max_outer=5, rel_tol=0.0, check_every=2, **ACCURATE)
    say(f"batch fixed 5 steps {dtype}")
    us, st, ts, As = d.dehaze_batch(ctx(), [dev(a) for a in arrs], params=p, want_t=True)
    for k, (arr, I) in enumerate(zip(arrs, I32)):
        ref_pr = o.prior(I)
        A = host(As[k]).astype(np.float64)
        assert np.array_equal(A, ref_pr["A"])
        assert np.max(np.abs(host(ts[k]) - ref_pr["t"])) <= 2.0 ** -24
        ref = o.solve(ref_pr["phi"], ref_pr["lam"], "picard", steps=5)
        err = np.max(np.abs(host(us[k]) - ref.u))
        say(f"  image {k} {arr.shape} max-abs {err:.3e} outer {st[k]['outer']}")
        assert err <= U_TOL
        assert st[k]["outer"] == 5
        # the one-image entry points run the same kernels on the same bits
        pr = d.dehaze_prior(ctx(), dev(arr), outputs=("t",))
        u1, st1 = d.dehaze_solve(ctx(), dev(arr), pr["t"], pr["A"], params=p)
        assert np.array_equal(host(u1), host(us[k]))
        assert st1["rel_residual"] == st[k]["rel_residual"]


def test_batch_to_tolerance_per_image_masks():
    require_gpu()
    import paper_2506_08793_amd as d
    sizes = [(24, 24), (40, 31), (17, 50), (33, 33)]
    arrs, I32 = _images(sizes, 600)
    p = d.dehaze_params_default(max_outer=4000, rel_tol=1e-5, inner_rtol=0.1, max_inner=10, check_every=16)
    say("batch to 1e-5")
    us, st, ts, As = d.dehaze_batch(ctx(), [dev(a) for a in arrs], params=p)
    outers = [s["outer"] for s in st]
    say(f"  outer steps per image {outers}")
    assert all(s["converged"] and s["status"] == 0 and s["rel_residual"] <= 1e-5 for s in st)
    assert len(set(outers)) > 1  # images stop independently
    for k, I in enumerate(I32):
        pr = o.prior(I)
        ref = o.solve(pr["phi"], pr["lam"], "picard", rel_tol=1e-10, max_steps=4000)
        _, floor = o.residual(ref.u.astype(np.float32).astype(np.float64), pr["phi"], pr["lam"])
        _, rho_u = o.residual(host(us[k]).astype(np.float64), pr["phi"], pr["lam"])
        dist = np.max(np.abs(host(us[k]) - ref.u))
        say(f"  image {k}: oracle rho(u) {rho_u:.3e} float32 floor {floor:.3e} max-abs vs converged {dist:.3e}")
        assert rho_u <= 2.0 * floor + 2e-5
        assert dist <= 1e-2


def test_batch_given_t_A_u0_and_graph_reuse():
    require_gpu()
    import paper_2506_08793_amd as d
    sizes = [(30, 20), (20, 45)]
    arrs, I32 = _images(sizes, 700)
    prs = [o.prior(I) for I in I32]
    t = [dev(pr["t"].astype(np.float32)) for pr in prs]
    A = [dev(pr["A"].astype(np.float32)) for pr in prs]
    rng = np.random.default_rng(3)
    u0 = []
    for pr in prs:
        u0.append(dev((pr["phi"] + rng.uniform(-0.3, 0.3, size=pr["phi"].shape)).astype(np.float32)))
    p = d.dehaze_params_default(max_outer=4, rel_tol=0.0, check_every=2, **ACCURATE)
    ws = d.binding._workspace(d.batch_workspace_bytes(sizes, p), "cuda")
    say("batch given t, A, u0 (twice)")
    us1, st1, _, _ = d.dehaze_batch(ctx(), [dev(a) for a in arrs], params=p, t=t, A=A, u0=u0, ws=ws)
    r1 = [host(u) for u in us1]
    us2, st2, _, _ = d.dehaze_batch(ctx(), [dev(a) for a in arrs], params=p, t=t, A=A, u0=u0, ws=ws)
    for k, pr in enumerate(prs):
        assert np.array_equal(r1[k], host(us2[k]))
        t32 = pr["t"].astype(np.float32)
        lam = o.adaptive_weight(t32.astype(np.float64))
        phi = o.reconstruction(I32[k], t32, pr["A"].astype(np.float32), o.DEFAULT.t0)
        ref = o.solve(phi, lam, "picard", steps=4, u0=host(u0[k]).astype(np.float64))
        assert np.max(np.abs(r1[k] - ref.u)) <= U_TOL


def test_batch_rejects_bad_arguments():
    require_gpu()
    import paper_2506_08793_amd as d
    arrs, _ = _images([(8, 8)], 800)
    with pytest.raises(d.DehazeError):
        d.dehaze_batch(ctx(), [dev(arrs[0])], params=d.dehaze_params_default(scheme=d.JACOBI))
    with pytest.raises(d.DehazeError):
        d.dehaze_batch(ctx(), [dev(arrs[0])], params=d.dehaze_params_default(inner_refine=-1))


@pytest.mark.parametrize("warm", [0, 2])
def test_batch_images_progress_independently(warm):
    # Default settings (tick loop): each image keeps its own BiCGSTAB
    # iteration count, so an image of a batch goes through exactly the steps
    # it goes through alone, whatever the other images need.  Sizes chosen so
    # that the images differ in outer steps and iterations per step.  The
    # strip height the batch's tuner picks for an image may differ from the
    # one it gets alone; the results do not depend on it (next test).
    require_gpu()
    import paper_2506_08793_amd as d
    sizes = [(96, 128), (40, 31), (200, 150), (1, 1)]
    arrs, _ = _images(sizes, 800)
    p = d.dehaze_params_default(max_outer=3000, rel_tol=1e-5, warm_start=warm)
    say(f"batch vs single, default settings, warm_start={warm}")
    us, st, _, _ = d.dehaze_batch(ctx(), [dev(a) for a in arrs], params=p)
    say(f"  outer {[s['outer'] for s in st]} inner {[s['inner'] for s in st]}")
    assert len({s["outer"] for s in st}) > 1
    for k, a in enumerate(arrs):
        u1, st1, _, _ = d.dehaze_batch(ctx(), [dev(a)], params=p)
        assert np.array_equal(host(u1[0]), host(us[k])), k
        for key in ("outer", "inner", "applications", "rel_residual", "rel_residual0", "converged", "restarts"):
            assert st1[0][key] == st[k][key], (k, key)


def test_batch_float64_output():
    # u_state = DEHAZE_U_F64: every image returns its float64 iterate, whose
    # float32 rounding is the float32 output and whose residual the stats give
    require_gpu()
    import paper_2506_08793_amd as d
    import torch
    arrs, _ = _images([(24, 24), (40, 31), (17, 50)], 650)
    imgs = [dev(a) for a in arrs]
    p = d.dehaze_params_default(max_outer=4000, rel_tol=1e-5)
    say("batch to 1e-5, float32 and float64 outputs")
    u32, st32, _, _ = d.dehaze_batch(ctx(), imgs, params=p)
    u64, st64, _, _ = d.dehaze_batch(ctx(), imgs, params=p.replace(u_state=d.U_F64))
    for k in range(len(imgs)):
        assert u64[k].dtype == torch.float64
        assert np.array_equal(host(u64[k]).astype(np.float32), host(u32[k]))
        assert st64[k]["converged"] and st64[k]["rel_residual_out"] == st64[k]["rel_residual"] <= 1e-5
        assert st64[k]["rel_residual"] == st32[k]["rel_residual"]


def test_strip_height_does_not_change_results():
    # The BiCGSTAB strip kernels sum their dot products per block of 16 rows
    # in a fixed order, so every strip height, forced or tuned, gives the same
    # iterates bit for bit: several column groups, a ragged last strip, and a
    # batch of uneven sizes.
    require_gpu()
    import paper_2506_08793_amd as d
    sizes = [(300, 517), (40, 31), (129, 70)]
    arrs, _ = _images(sizes, 900)
    imgs = [dev(a) for a in arrs]
    base = d.dehaze_params_default(max_outer=6, rel_tol=0.0)
    ref = None
    for rows in (16, 32, 48, 64, 128, 256, 0):
        say(f"strip rows {rows}")
        us, st, _, _ = d.dehaze_batch(ctx(), imgs, params=base.replace(krylov_rows=rows))
        got = [host(u) for u in us]
        if ref is None:
            ref = (got, st)
            continue
        for k in range(len(sizes)):
            assert np.array_equal(got[k], ref[0][k]), (rows, k)
            for key in ("outer", "inner", "rel_residual", "rel_residual_out"):
                assert st[k][key] == ref[1][k][key], (rows, k, key)
    chosen, tuned = d.dehaze_batch_strip_rows(ctx(), sizes, base)
    say(f"  tuned strip rows {chosen}")
    assert tuned and all(r in (16, 32, 64, 128, 256) for r in chosen)
