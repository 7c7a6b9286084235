"""Pins of the oracle's accelerated lagged-diffusivity iteration (nonlinear
GMRES over earlier iterates): the mixing least squares against a library
solver, exactness of the mixed residual where the residual map is affine,
reduction to the plain iteration at depth 0, and the common fixed point."""
import numpy as np

import synth
from oracle import dehaze_ref as o

P = o.DEFAULT


def _problem(H, W, seed):
    img = synth.hazy_image(H, W, seed, beta_haze=1.0, occlusion=True)
    pr = o.prior(img["I"], P)
    return pr["phi"], pr["lam"]


def test_mix_coefficients_are_the_least_squares_solution():
    # the normal equations with their tiny shift solve the same problem as a
    # QR/SVD least-squares routine, and the mixed residual is orthogonal to
    # every residual difference
    rng = np.random.default_rng(3)
    shape = (3, 9, 11)
    rt = rng.normal(size=shape)
    R = [rt + rng.normal(scale=0.3, size=shape) for _ in range(4)]
    U = [rng.normal(size=shape) for _ in range(4)]
    ut = rng.normal(size=shape)
    um, rm, b = o.ngmres_mix(ut, rt, U, R)
    A = np.stack([(rt - Rj).reshape(-1) for Rj in R], axis=1)
    b_ref, *_ = np.linalg.lstsq(A, -rt.reshape(-1), rcond=None)
    assert np.max(np.abs(b - b_ref)) <= 1e-8 * np.max(np.abs(b_ref))
    assert np.max(np.abs(A.T @ rm.reshape(-1))) <= 1e-8 * np.linalg.norm(rt)
    # the mixed iterate is the same affine combination as the mixed residual
    assert np.allclose(um, (1 + b.sum()) * ut - sum(bj * Uj for bj, Uj in zip(b, U)), atol=1e-12)


def test_mixed_residual_is_exact_for_an_affine_residual():
    # with D = 1 (no edge preservation) r(u) = Phi - L u is affine in u, so the
    # combination of residuals is the residual of the combination of iterates
    q = o.with_params(edge_preserving=False)
    phi, lam = _problem(10, 13, 4)
    rng = np.random.default_rng(5)
    iters = [phi + rng.normal(size=phi.shape) for _ in range(4)]
    res = [o.residual(u, phi, lam, q)[0] for u in iters]
    um, rm, _ = o.ngmres_mix(iters[-1], res[-1], iters[:-1], res[:-1])
    r_true, _ = o.residual(um, phi, lam, q)
    assert np.max(np.abs(rm - r_true)) <= 1e-10 * np.max(np.abs(r_true))
    # and it is the smallest such residual: no random combination does better
    for _ in range(20):
        c = rng.normal(size=3)
        uc = iters[-1] + sum(cj * (iters[-1] - Uj) for cj, Uj in zip(c, iters[:-1]))
        assert np.linalg.norm(o.residual(uc, phi, lam, q)[0]) >= np.linalg.norm(rm) * (1 - 1e-12)


def test_depth_zero_is_the_plain_iteration():
    phi, lam = _problem(12, 10, 6)
    a = o.solve(phi, lam, "picard", P, steps=5)
    b = o.ngmres_solve(phi, lam, P, depth=0, steps=5)
    assert np.max(np.abs(a.u - b.u)) <= 1e-10 * np.max(np.abs(a.u))
    assert np.allclose(a.rho, b.rho, rtol=1e-9, atol=0)


def test_accelerated_iteration_reaches_the_same_fixed_point_in_fewer_steps():
    # both iterations stop at rho <= 1e-9 and then lie within what two such
    # iterates may differ by; the mixed one needs far fewer steps
    phi, lam = _problem(20, 24, 7)
    plain = o.solve(phi, lam, "picard", P, rel_tol=1e-9, max_steps=3000)
    acc = o.ngmres_solve(phi, lam, P, depth=5, rel_tol=1e-9, max_steps=3000)
    assert plain.rho[-1] <= 1e-9 and acc.rho[-1] <= 1e-9
    assert acc.steps < 0.6 * plain.steps, (acc.steps, plain.steps)
    assert np.max(np.abs(acc.u - plain.u)) <= 1e-5 * np.max(np.abs(plain.u))
