"""Pins of the oracle's iterations (Appendix A-1) and of the lagged-diffusivity
fixed point: direct vs library iterative solves, manufactured solutions,
fixed-point consistency and the explicit step bound."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import dehaze_ref as o

P = o.DEFAULT


def _problem(H, W, seed):
    img = synth.hazy_image(H, W, seed, beta_haze=1.0)
    pr = o.prior(img["I"], P)
    return pr["phi"], pr["lam"]


def test_explicit_and_jacobi_steps_match_matrix_form():
    phi, lam = _problem(10, 12, 1)
    rng = np.random.default_rng(2)
    u = phi + rng.uniform(-1, 1, size=phi.shape)
    w = o.gaussian_taps(P.sigma, P.g_radius)
    Dx, Dy = o.face_coefficients(u, P)
    ue = o.explicit_step(u, phi, lam, P)
    uj = o.jacobi_sweep(u, phi, lam, P)
    for c in range(3):
        L = o.assemble_operator(Dx[c], Dy[c], lam, w, P)
        r = phi[c].reshape(-1) - L @ u[c].reshape(-1)
        assert np.max(np.abs(ue[c].reshape(-1) - (u[c].reshape(-1) + P.tau * r))) < 1e-11
        want = u[c].reshape(-1) + P.theta * r / L.diagonal()
        assert np.max(np.abs(uj[c].reshape(-1) - want)) < 1e-11


def test_picard_step_direct_vs_dense_and_iterative():
    phi, lam = _problem(12, 11, 3)
    u = o.picard_step(phi, phi, lam, P)
    w = o.gaussian_taps(P.sigma, P.g_radius)
    Dx, Dy = o.face_coefficients(phi, P)
    for c in range(3):
        L = o.assemble_operator(Dx[c], Dy[c], lam, w, P)
        dense = np.linalg.solve(L.toarray(), phi[c].reshape(-1))
        assert np.max(np.abs(dense - u[c].reshape(-1))) < 1e-9 * np.abs(dense).max()
        it, info = spla.gmres(L, phi[c].reshape(-1), rtol=1e-13, atol=0, restart=200, maxiter=50)
        assert info == 0
        assert np.max(np.abs(it - u[c].reshape(-1))) < 1e-7 * np.abs(dense).max()


def test_manufactured_solution_is_a_fixed_point_and_attracts():
    # choose u_m, define Phi := L(D(u_m)) u_m; the residual vanishes at u_m and
    # the lagged-diffusivity iteration started nearby returns to it
    H, W = 14, 13
    yy, xx = np.mgrid[0:H, 0:W]
    um = np.stack([2.0 + np.sin(xx / 3.0 + c) * np.cos(yy / 4.0) for c in range(3)])
    lam = 0.5 * np.exp(-3.0 * (1 - np.linspace(0.2, 0.9, H * W).reshape(H, W)))
    w = o.gaussian_taps(P.sigma, P.g_radius)
    Dx, Dy = o.face_coefficients(um, P)
    phi = o.operator_apply(um, Dx, Dy, lam, w, P)
    _, rho = o.residual(um, phi, lam, P)
    assert rho < 1e-14
    rng = np.random.default_rng(0)
    res = o.solve(phi, lam, "picard", P, rel_tol=1e-10, u0=um + 0.05 * rng.standard_normal(um.shape),
                  max_steps=2000)
    assert res.rho[-1] <= 1e-10
    assert np.max(np.abs(res.u - um)) < 1e-7


@pytest.mark.slow
def test_fixed_point_consistency_of_all_three_schemes():
    phi, lam = _problem(16, 16, 4)
    res = o.solve(phi, lam, "picard", P, rel_tol=1e-12, max_steps=3000)
    us = res.u
    assert res.rho[-1] <= 1e-12
    scale = np.abs(us).max()
    for step in (o.explicit_step, o.jacobi_sweep, o.picard_step):
        assert np.max(np.abs(step(us, phi, lam, P) - us)) < 1e-8 * scale


def test_picard_decreases_residual_on_small_workload():
    img = synth.small_image()
    pr = o.prior(img["I"], P)
    res = o.solve(pr["phi"], pr["lam"], "picard", P, steps=8)
    assert res.rho[-1] < 0.2 * res.rho[0]


def test_explicit_step_bound_closed_form_and_conservative():
    # Appendix A-1: tau < 2 / (||D Laplacian|| + lambda M); with D <= 1/eps,
    # ||Laplacian|| <= 8, lambda <= lambda0 and M = 1 the bound is 2/(8/eps + lambda0).
    tau_max = o.explicit_step_bound(P)
    assert abs(tau_max - 2.0 / (8000.0 + 0.5)) < 1e-18
    assert tau_max < P.tau / 500          # the paper's tau = 0.2 is far above it
    # the bound is conservative: every eigenvalue of the frozen operator lies
    # below 8/eps + lambda0 in modulus, so I - tau L is a contraction for
    # symmetric L when tau < tau_max
    H, W = 8, 8
    rng = np.random.default_rng(5)
    u = rng.uniform(0, 1e-4, size=(1, H, W))      # flat u: D close to 1/eps
    lam = np.full((H, W), P.lambda0)
    w = o.gaussian_taps(P.sigma, P.g_radius)
    Dx, Dy = o.face_coefficients(u, P)
    L = o.assemble_operator(Dx[0], Dy[0], lam, w, P).toarray()
    ev = np.linalg.eigvalsh(0.5 * (L + L.T))
    assert ev.max() <= 8.0 / P.eps + P.lambda0
    assert np.max(np.abs(1.0 - 0.99 * tau_max * ev)) < 1.0
    assert np.max(np.abs(1.0 - P.tau * ev)) > 1.0


def test_solve_stops_on_tolerance_and_counts():
    phi, lam = _problem(8, 9, 6)
    r = o.solve(phi, lam, "jacobi", P, steps=5)
    assert r.steps == 5 and len(r.rho) == 6
    r2 = o.solve(phi, lam, "picard", P, rel_tol=1e-3, max_steps=1000)
    assert r2.rho[-1] <= 1e-3 and all(x > 1e-3 for x in r2.rho[:-1])
