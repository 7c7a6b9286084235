"""GPU sweeps (Appendix A-1 explicit update and its Jacobi-scaled form) and
the residual of the main PDE vs the FP64 oracle, on the same float32 t and A."""
import numpy as np
import pytest

import synth
from gpu_util import ctx, dev, host, require_gpu, say
from oracle import dehaze_ref as o

pytestmark = pytest.mark.gpu

# max-abs bound on u in units where I lies in [0, 1]
U_TOL = 1e-4
# The residual of a float32 iterate is formed in float32 per pixel (terms of
# size |Phi|, rounding 2^-24 each, a few dozen of them) and summed in float64:
# its relative value carries an absolute error of a few 1e-7.
RHO_ABS = 4e-6


def rho_close(a, b, rtol):
    return abs(a - b) <= rtol * abs(b) + RHO_ABS


def _inputs(H, W, seed, beta=(0.5, 2.0)):
    img = synth.hazy_image(H, W, seed, beta_haze=beta, occlusion=True)
    pr = o.prior(img["I"])
    t32 = pr["t"].astype(np.float32)
    A32 = pr["A"].astype(np.float32)
    lam = o.adaptive_weight(t32.astype(np.float64))
    phi = o.reconstruction(img["I"], t32, A32, o.DEFAULT.t0)
    return img["I"], t32, A32, lam, phi


def _gpu_solve(I, t32, A32, **kw):
    import paper_2506_08793_amd as d
    p = d.dehaze_params_default(**kw)
    u, st = d.dehaze_solve(ctx(), dev(I), dev(t32), dev(A32), params=p)
    return host(u), st


@pytest.mark.parametrize("H,W,seed,n", [(64, 64, 1000, 200), (1, 1, 3, 20), (3, 2, 4, 20), (37, 53, 5, 60),
                                        (17, 130, 6, 40), (100, 67, 7, 30), (16, 64, 8, 25)])
def test_jacobi_parity(H, W, seed, n):
    require_gpu()
    I, t32, A32, lam, phi = _inputs(H, W, seed)
    say(f"jacobi H={H} W={W} n={n}")
    u, st = _gpu_solve(I, t32, A32, scheme=1, max_outer=n, rel_tol=0.0)
    ref = o.solve(phi, lam, "jacobi", steps=n)
    err = np.max(np.abs(u - ref.u))
    say(f"  max-abs {err:.3e}  rho gpu {st['rel_residual']:.6e} oracle {ref.rho[-1]:.6e}")
    assert err <= U_TOL
    assert st["outer"] == n and st["applications"] == n
    assert rho_close(st["rel_residual0"], ref.rho[0], 1e-5)
    assert rho_close(st["rel_residual"], ref.rho[-1], 1e-4)


@pytest.mark.parametrize("n", [1, 2])
def test_explicit_parity_few_steps(n):
    # the tau = 0.2 update is unstable (its step bound is ~2.5e-4), so only
    # the first steps are reproducible in float32
    require_gpu()
    I, t32, A32, lam, phi = _inputs(64, 64, 1000, beta=1.0)
    say(f"explicit n={n}")
    u, st = _gpu_solve(I, t32, A32, scheme=0, max_outer=n, rel_tol=0.0)
    ref = o.solve(phi, lam, "explicit", steps=n)
    assert np.max(np.abs(u - ref.u)) <= U_TOL


def test_jacobi_from_given_start_and_ablations():
    require_gpu()
    I, t32, A32, lam, phi = _inputs(40, 50, 9)
    rng = np.random.default_rng(1)
    u0 = (phi + rng.uniform(-0.5, 0.5, size=phi.shape)).astype(np.float32)
    import paper_2506_08793_amd as d
    for flags in ({}, {"nonlocal_term": 0}, {"edge_preserving": 0}, {"adaptive": 0}):
        say(f"jacobi u0 flags={flags}")
        p = d.dehaze_params_default(scheme=1, max_outer=25, rel_tol=0.0, **flags)
        u, st = d.dehaze_solve(ctx(), dev(I), dev(t32), dev(A32), params=p, u0=dev(u0))
        q = o.with_params(**{k: bool(v) for k, v in flags.items()})
        lam_q = o.adaptive_weight(t32.astype(np.float64), q)
        ref = o.solve(phi, lam_q, "jacobi", q, steps=25, u0=u0.astype(np.float64))
        assert np.max(np.abs(host(u) - ref.u)) <= U_TOL


def test_jacobi_stops_on_tolerance():
    require_gpu()
    I, t32, A32, lam, phi = _inputs(24, 24, 10)
    say("jacobi rel_tol")
    u, st = _gpu_solve(I, t32, A32, scheme=1, max_outer=400, rel_tol=0.9, check_every=4)
    assert st["converged"] and st["rel_residual"] <= 0.9 and st["outer"] % 4 == 0
    assert st["rel_residual_out"] == st["rel_residual"]  # float32 iterate: the output itself
    _, rho = o.residual(u.astype(np.float64), phi, lam)
    assert rho_close(st["rel_residual"], rho, 1e-5)
    # not reachable: ENOTCONV is returned as a status, u holds the last iterate
    u2, st2 = _gpu_solve(I, t32, A32, scheme=1, max_outer=8, rel_tol=1e-9, check_every=4)
    assert not st2["converged"] and st2["status"] == -4 and st2["outer"] == 8


@pytest.mark.parametrize("H,W", [(1, 1), (7, 9), (64, 64), (33, 200)])
def test_residual_entry_point(H, W):
    require_gpu()
    import paper_2506_08793_amd as d
    I, t32, A32, lam, phi = _inputs(H, W, 40 + H)
    rng = np.random.default_rng(H * W)
    u = (phi + rng.uniform(-1, 1, size=phi.shape)).astype(np.float32)
    say(f"residual H={H} W={W}")
    rho, r = d.dehaze_residual(ctx(), dev(u), dev(phi.astype(np.float32)), dev(lam.astype(np.float32)),
                               want_r=True)
    r_ref, rho_ref = o.residual(u.astype(np.float64), phi.astype(np.float32).astype(np.float64),
                                lam.astype(np.float32).astype(np.float64))
    assert rho_close(rho, rho_ref, 1e-5)
    scale = np.abs(r_ref).max() + 1.0
    assert np.max(np.abs(host(r) - r_ref)) <= 1e-5 * scale


def test_jacobi_full_megapixel_workload():
    # the 1024x1024 workload in the configuration the benchmark times (the
    # tuned launch shape, all 200 sweeps); the oracle follows every sweep
    # element by element (about a minute of float64 numpy)
    require_gpu()
    I, t32, A32, lam, phi = _inputs(1024, 1024, 2000)
    say("jacobi 1024x1024 n=200")
    u, st = _gpu_solve(I, t32, A32, scheme=1, max_outer=200, rel_tol=0.0)
    ref = o.solve(phi, lam, "jacobi", steps=200)
    err = np.max(np.abs(u - ref.u))
    say(f"  max-abs {err:.3e} rho gpu {st['rel_residual']:.6e} oracle {ref.rho[-1]:.6e}")
    assert err <= U_TOL
    assert rho_close(st["rel_residual"], ref.rho[-1], 1e-4)


@pytest.mark.parametrize("cols", [1, 2])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("H,W,seed", [(37, 53, 60), (130, 67, 61), (1, 1, 62), (5, 300, 63), (64, 64, 1000)])
def test_sweeps_per_launch_parity_and_invariance(k, cols, H, W, seed):
    # K sweeps pipelined in one launch: same values as the oracle's sweeps, and
    # bit for bit the same as one sweep per launch with one column per lane
    require_gpu()
    I, t32, A32, lam, phi = _inputs(H, W, seed)
    n = 13
    say(f"jacobi K={k} C={cols} H={H} W={W}")
    u, st = _gpu_solve(I, t32, A32, scheme=1, max_outer=n, rel_tol=0.0, sweeps_per_launch=k, lane_columns=cols)
    u1, _ = _gpu_solve(I, t32, A32, scheme=1, max_outer=n, rel_tol=0.0, sweeps_per_launch=1, lane_columns=1)
    assert np.array_equal(u, u1)
    # strip heights, including ones that are not a multiple of the 4-row
    # unroll and ones taller than the image
    for rows in (3, 6, 13, 40, 300):
        us, _ = _gpu_solve(I, t32, A32, scheme=1, max_outer=n, rel_tol=0.0, sweeps_per_launch=k, strip_rows=rows,
                           lane_columns=cols)
        assert np.array_equal(us, u1), rows
    ref = o.solve(phi, lam, "jacobi", steps=n)
    assert np.max(np.abs(u - ref.u)) <= U_TOL
    # the tau = 0.2 update amplifies rounding by up to tau * 8 / eps per step,
    # so only its first step is compared with the oracle on sharp-edged input;
    # two steps in one launch must equal two launches of one step exactly
    ue1, _ = _gpu_solve(I, t32, A32, scheme=0, max_outer=1, rel_tol=0.0, sweeps_per_launch=1)
    assert np.max(np.abs(ue1 - o.solve(phi, lam, "explicit", steps=1).u)) <= U_TOL
    ue2, _ = _gpu_solve(I, t32, A32, scheme=0, max_outer=2, rel_tol=0.0, sweeps_per_launch=min(k, 2),
                        lane_columns=cols)
    ue2b, _ = _gpu_solve(I, t32, A32, scheme=0, max_outer=2, rel_tol=0.0, sweeps_per_launch=1, lane_columns=1)
    assert np.array_equal(ue2, ue2b)


def test_other_gaussian_radius_uses_tile_kernel():
    require_gpu()
    import paper_2506_08793_amd as d
    I, t32, A32, lam, phi = _inputs(41, 70, 64)
    say("jacobi g_radius=3")
    u, st = _gpu_solve(I, t32, A32, scheme=1, max_outer=20, rel_tol=0.0, g_radius=3, sigma=2.0)
    q = o.with_params(g_radius=3, sigma=2.0)
    ref = o.solve(phi, lam, "jacobi", q, steps=20)
    assert np.max(np.abs(u - ref.u)) <= U_TOL
    assert d.dehaze_sweep_shape(ctx(), 41, 70, d.JACOBI) == (0, 0, 0)  # R != 2: tile kernel, nothing tuned


def test_autotuned_shape_is_recorded():
    require_gpu()
    import paper_2506_08793_amd as d
    I, t32, A32, lam, phi = _inputs(200, 150, 65)
    u, st = _gpu_solve(I, t32, A32, scheme=1, max_outer=7, rel_tol=0.0)
    k, srows, cols = d.dehaze_sweep_shape(ctx(), 200, 150, d.JACOBI)
    say(f"  autotuned K={k} S={srows} C={cols}")
    assert 1 <= k <= 4 and 4 <= srows <= 131 and cols in (1, 2)
    assert np.max(np.abs(u - o.solve(phi, lam, "jacobi", steps=7).u)) <= U_TOL
