"""GPU lagged-diffusivity solve (Picard outer steps, BiCGSTAB corrections) vs
the oracle's exact Picard steps (sparse LU per step), on the same float32 t, A."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import ctx, dev, host, require_gpu, say, ulp32
from oracle import dehaze_ref as o

pytestmark = pytest.mark.gpu

U_TOL = 1e-4
# absolute slack on a relative residual formed from float32 Phi and lambda
# (a few 1e-7 per pixel, summed in float64)
RHO_ABS = 4e-6


def _inputs(H, W, seed, beta=1.0, occlusion=False):
    img = synth.hazy_image(H, W, seed, beta_haze=beta, occlusion=occlusion)
    pr = o.prior(img["I"])
    t32 = pr["t"].astype(np.float32)
    A32 = pr["A"].astype(np.float32)
    lam = o.adaptive_weight(t32.astype(np.float64))
    phi = o.reconstruction(img["I"], t32, A32, o.DEFAULT.t0)
    return img["I"], t32, A32, lam, phi


def _solve(I, t32, A32, u0=None, **kw):
    import paper_2506_08793_amd as d
    p = d.dehaze_params_default(scheme=d.PICARD_KRYLOV, **kw)
    u, st = d.dehaze_solve(ctx(), dev(I), dev(t32), dev(A32), params=p,
                           u0=None if u0 is None else dev(u0.astype(np.float32)))
    return host(u), st


def test_picard_50_steps_small_workload():
    # 64x64 workload: 50 lagged-diffusivity steps with tight inner solves
    require_gpu()
    I, t32, A32, lam, phi = _inputs(64, 64, 1000)
    say("picard 64x64 50 steps")
    u, st = _solve(I, t32, A32, max_outer=50, rel_tol=0.0, inner_rtol=1e-4, max_inner=200, inner_refine=3)
    ref = o.solve(phi, lam, "picard", steps=50)
    err = np.max(np.abs(u - ref.u))
    say(f"  max-abs {err:.3e} rho gpu {st['rel_residual']:.6e} oracle {ref.rho[-1]:.6e} inner {st['inner']}")
    assert err <= U_TOL
    assert st["outer"] == 50
    assert abs(st["rel_residual"] - ref.rho[-1]) <= 1e-3 * ref.rho[-1] + 1e-6
    assert abs(st["rel_residual0"] - ref.rho[0]) <= 1e-6 * ref.rho[0]


@pytest.mark.parametrize("H,W,seed,n", [(1, 1, 3, 3), (3, 2, 4, 4), (37, 53, 5, 6), (17, 130, 6, 5),
                                        (100, 67, 7, 4)])
def test_picard_ragged_shapes(H, W, seed, n):
    require_gpu()
    I, t32, A32, lam, phi = _inputs(H, W, seed, beta=(0.5, 2.0), occlusion=True)
    say(f"picard H={H} W={W} n={n}")
    u, st = _solve(I, t32, A32, max_outer=n, rel_tol=0.0, inner_rtol=1e-4, max_inner=200, inner_refine=3)
    ref = o.solve(phi, lam, "picard", steps=n)
    err = np.max(np.abs(u - ref.u))
    say(f"  max-abs {err:.3e}")
    assert err <= U_TOL


def test_picard_from_given_start_and_ablations():
    require_gpu()
    I, t32, A32, lam, phi = _inputs(30, 41, 8)
    rng = np.random.default_rng(2)
    u0 = phi + rng.uniform(-0.5, 0.5, size=phi.shape)
    for flags in ({}, {"nonlocal_term": 0}, {"edge_preserving": 0}, {"adaptive": 0}):
        say(f"picard u0 flags={flags}")
        u, st = _solve(I, t32, A32, u0=u0, max_outer=4, rel_tol=0.0, inner_rtol=1e-4, max_inner=200, inner_refine=3, **flags)
        q = o.with_params(**{k: bool(v) for k, v in flags.items()})
        lam_q = o.adaptive_weight(t32.astype(np.float64), q)
        ref = o.solve(phi, lam_q, "picard", q, steps=4, u0=u0.astype(np.float32).astype(np.float64))
        err = np.max(np.abs(u - ref.u))
        scale = max(1.0, np.max(np.abs(ref.u)))
        say(f"  max-abs {err:.3e} max|u| {scale:.1f}")
        if flags:
            # without lambda G (or with D = 1) u grows to O(1e3) and the
            # operator loses its zeroth-order term; a float32 u alone carries
            # 2^-24 |u|, so the bound is relative to |u| there
            assert err <= 1e-3 * scale
        else:
            assert err <= U_TOL


def test_picard_reaches_tolerance():
    # residual-terminated solve: the float64 residual the library reports must
    # be <= 1e-5; the oracle checks the float32 output against the float32
    # rounding floor of its own converged solution, and reports the distance
    require_gpu()
    I, t32, A32, lam, phi = _inputs(32, 32, 12)
    say("picard 32x32 to 1e-5")
    u, st = _solve(I, t32, A32, max_outer=3000, rel_tol=1e-5, inner_rtol=0.1, max_inner=10, check_every=16)
    say(f"  {st}")
    assert st["converged"] and st["status"] == 0 and st["rel_residual"] <= 1e-5
    assert st["outer"] % 16 != 0 or st["outer"] > 0
    _, rho_gpu_u = o.residual(u.astype(np.float64), phi, lam)
    ref = o.solve(phi, lam, "picard", rel_tol=1e-10, max_steps=3000)
    _, floor = o.residual(ref.u.astype(np.float32).astype(np.float64), phi, lam)
    say(f"  oracle rho of float32 output {rho_gpu_u:.3e}, float32 floor {floor:.3e}, "
        f"max-abs vs converged {np.max(np.abs(u - ref.u)):.3e}")
    assert rho_gpu_u <= 2.0 * floor + 2e-5
    # the residual the library reports for its float32 output is that of u
    assert abs(rho_gpu_u - st["rel_residual_out"]) <= 1e-4 * rho_gpu_u + RHO_ABS
    assert np.max(np.abs(u - ref.u)) <= 1e-2


def test_picard_not_converged_status():
    require_gpu()
    I, t32, A32, lam, phi = _inputs(16, 16, 13)
    say("picard ENOTCONV")
    u, st = _solve(I, t32, A32, max_outer=3, rel_tol=1e-12, check_every=1)
    assert not st["converged"] and st["status"] == -4 and st["outer"] == 3
    assert np.all(np.isfinite(u))


def test_stall_watch_restart_and_stop():
    # One-step window: a tolerance solve from Phi stops at its first step that
    # does not halve rho (stalled, DEHAZE_ENOTCONV); from a given start it
    # first restarts from Phi, after which it is the cold solve step for step
    # and stops at the same point with the same u, bit for bit.
    require_gpu()
    I, t32, A32, lam, phi = _inputs(48, 40, 14, beta=1.0, occlusion=True)
    rng = np.random.default_rng(5)
    u0 = phi + rng.normal(0.0, 0.5, size=phi.shape)
    say("picard stall watch (window 1)")
    kw = dict(max_outer=3000, rel_tol=1e-5, check_every=16)
    uc, stc = _solve(I, t32, A32, stall_window=1, **kw)
    uw, stw = _solve(I, t32, A32, u0=u0, stall_window=1, **kw)
    say(f"  cold {stc}\n  from u0 {stw}")
    assert stc["stalled"] == 1 and stc["restarts"] == 0 and not stc["converged"] and stc["status"] == -4
    assert stc["outer"] < 200 and stc["rel_residual"] > 1e-5
    assert stw["restarts"] == 1 and stw["stalled"] == 1 and stw["outer"] > stc["outer"]
    assert np.array_equal(uw, uc)
    # the default window lets the same solves converge; a zero window never acts
    ud, std = _solve(I, t32, A32, **kw)
    assert std["converged"] and std["stalled"] == 0 and std["restarts"] == 0
    un, stn = _solve(I, t32, A32, u0=u0, stall_window=0, **kw)
    assert stn["restarts"] == 0 and stn["stalled"] == 0


def test_warm_starts_reach_the_cold_solution():
    # 512x512 window (seed 9103, held out), whose cold solve crosses a long
    # plateau near rho = 4e-5: from the analytic start and from the network
    # the solve converges too, without a restart, to within the distance two
    # rho <= 1e-5 iterates may lie apart.
    require_gpu()
    import paper_2506_08793_amd as d
    from paper_2506_08793_amd import warmstart
    warmstart.load(ctx(), warmstart.default_weights_path())
    img = synth.hazy_window(512, 512, 9103)
    I = dev(img["I"])
    pr = d.dehaze_prior(ctx(), I, outputs=("t",))
    say("picard 512x512 window 9103 cold / analytic / network")
    out = {}
    for warm in (0, 2, 1):
        p = d.dehaze_params_default(max_outer=4000, rel_tol=1e-5, warm_start=warm)
        u, st = d.dehaze_solve(ctx(), I, pr["t"], pr["A"], params=p)
        say(f"  warm_start={warm}: {st}")
        assert st["converged"] and st["stalled"] == 0 and st["restarts"] == 0
        out[warm] = host(u)
    for warm in (2, 1):
        assert np.max(np.abs(out[warm] - out[0])) <= 1e-2 * max(1.0, np.max(np.abs(out[0])))


def test_picard_full_size_1080p():
    # The 1080p workload of the images/s figure (held-out seed 7000), default
    # settings.  The float64 iterate meets rel_tol = 1e-5; the returned float32
    # u carries the rounding floor of float32 (u near 32, flux slope up to
    # 1/eps): the library reports that residual too, the oracle's float64
    # residual of the returned u must agree with it, and a further random
    # half-ulp perturbation of u must not lower it (u is as close to the
    # iterate as float32 allows, not merely near it).
    require_gpu()
    import paper_2506_08793_amd as d
    img = synth.hazy_image(1080, 1920, 7000, beta_haze=(0.5, 2.5), occlusion=True)
    say("picard 1080p to 1e-5 (defaults)")
    I = dev(img["I"])
    pg = d.dehaze_prior(ctx(), I, outputs=("t",))
    u, st = d.dehaze_solve(ctx(), I, pg["t"], pg["A"], params=d.dehaze_params_default())
    say(f"  {st}")
    assert st["converged"] and st["rel_residual"] <= 1e-5 and st["stalled"] == 0
    pr = o.prior(img["I"])
    uh = host(u).astype(np.float64)
    assert np.all(np.isfinite(uh))
    _, rho = o.residual(uh, pr["phi"], pr["lam"])
    rng = np.random.default_rng(7)
    nudge = np.where(rng.random(uh.shape) < 0.5, -0.5, 0.5) * ulp32(uh)
    _, rho_nudged = o.residual(uh + nudge, pr["phi"], pr["lam"])
    say(f"  oracle rho of the float32 output {rho:.3e}, library {st['rel_residual_out']:.3e}, "
        f"after a half-ulp nudge {rho_nudged:.3e}")
    assert abs(rho - st["rel_residual_out"]) <= 1e-4 * rho + RHO_ABS
    assert st["rel_residual"] <= rho <= rho_nudged


def test_picard_full_size_1080p_float64_output():
    # The same workload with u returned in float64 (u_state = DEHAZE_U_F64):
    # the caller now holds the iterate the tolerance was tested on, so the
    # oracle's float64 residual of the returned u (on the float32 Phi and
    # lambda the library formed) meets rel_tol and equals the reported value
    # up to summation order; rounding it to float32 gives the float32 output.
    require_gpu()
    import paper_2506_08793_amd as d
    img = synth.hazy_image(1080, 1920, 7000, beta_haze=(0.5, 2.5), occlusion=True)
    say("picard 1080p to 1e-5, float64 output")
    I = dev(img["I"])
    pg = d.dehaze_prior(ctx(), I, outputs=("t",))
    p64 = d.dehaze_params_default(u_state=d.U_F64)
    u64, st = d.dehaze_solve(ctx(), I, pg["t"], pg["A"], params=p64)
    say(f"  {st}")
    assert u64.dtype == torch.float64
    assert st["converged"] and st["rel_residual"] <= 1e-5 and st["rel_residual_out"] == st["rel_residual"]
    t32, A32 = host(pg["t"]), host(pg["A"])
    lam32 = o.adaptive_weight(t32.astype(np.float64)).astype(np.float32).astype(np.float64)
    phi32 = o.reconstruction(img["I"], t32, A32, o.DEFAULT.t0).astype(np.float32).astype(np.float64)
    _, rho = o.residual(host(u64), phi32, lam32)
    say(f"  oracle rho of the float64 output {rho:.6e}, library {st['rel_residual']:.6e}")
    assert rho <= 1e-5 * (1 + 1e-9)
    assert abs(rho - st["rel_residual"]) <= 1e-9 * rho
    u32, _ = d.dehaze_solve(ctx(), I, pg["t"], pg["A"], params=d.dehaze_params_default(), stats=False)
    assert np.array_equal(host(u64).astype(np.float32), host(u32))


@pytest.mark.parametrize("scheme", [1, 2])
def test_float64_output_is_the_iterate(scheme):
    # float32 output = the float64 output rounded (lagged diffusivity, whose
    # iterate is float64); the sweep schemes iterate in float32 and widen it
    require_gpu()
    import paper_2506_08793_amd as d
    I, t32, A32, lam, phi = _inputs(37, 53, 15, beta=(0.5, 2.0), occlusion=True)
    kw = dict(scheme=scheme, max_outer=12, rel_tol=0.0)
    say(f"float64 output scheme {scheme}")
    u32, st32 = d.dehaze_solve(ctx(), dev(I), dev(t32), dev(A32), params=d.dehaze_params_default(**kw))
    u64, st64 = d.dehaze_solve(ctx(), dev(I), dev(t32), dev(A32),
                               params=d.dehaze_params_default(u_state=d.U_F64, **kw))
    a32, a64 = host(u32), host(u64)
    assert a64.dtype == np.float64
    if scheme == 2:
        assert np.array_equal(a64.astype(np.float32), a32)
    else:
        assert np.array_equal(a64, a32.astype(np.float64))
    assert st64["rel_residual"] == st32["rel_residual"]
