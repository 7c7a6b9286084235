"""Pins of the oracle's operators: the Gaussian G (Section II-C, Appendix A-2),
the face-centred diffusion term (Appendix A-2), the assembled operator and
the structural facts of Section III (weak form, assumptions, coercivity)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import dehaze_ref as o

P = o.DEFAULT


def _rand_field(seed, C, H, W, scale=5.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, scale, size=(C, H, W))


def test_gaussian_taps_properties():
    for sigma in (1.5, 2.0):
        w = o.gaussian_taps(sigma, 2)
        assert len(w) == 5 and abs(w.sum() - 1.0) < 1e-15
        assert np.array_equal(w, w[::-1])
        assert abs(w[3] / w[2] - np.exp(-1.0 / (2 * sigma * sigma))) < 1e-15


def test_gaussian_taps_literal_values():
    # Section II-C's kernel exp(-a^2 / 2 sigma^2) on a = -2..2 (Appendix A-2's
    # 5x5 window), taps scaled to sum 1.  The numbers below were evaluated in
    # 40-digit decimal arithmetic, independently of numpy's exp, at the
    # workloads' sigma = 1.5 and the paper's sigma = 2.0; every tap is pinned,
    # so a wrong exponent (|a| for a^2, a missing factor 2) fails on the outer
    # taps even where the sum and the symmetry still hold.
    want = {
        1.5: [0.12007838424321348, 0.23388075658535030, 0.29208171834287245,
              0.23388075658535030, 0.12007838424321348],
        2.0: [0.15246914402033735, 0.22184129554377692, 0.25137912087177145,
              0.22184129554377692, 0.15246914402033735],
    }
    for sigma, w_lit in want.items():
        w = o.gaussian_taps(sigma, 2)
        assert np.max(np.abs(w - np.array(w_lit))) <= 2e-16, (sigma, w)


def test_gaussian_delta_response_and_library():
    w = o.gaussian_taps(1.5, 2)
    d = np.zeros((11, 13))
    d[5, 6] = 1.0
    g = o.gaussian_apply(d, w)
    assert np.allclose(g[3:8, 4:9], np.outer(w, w), rtol=0, atol=1e-17)
    assert np.count_nonzero(g) == 25
    u = _rand_field(1, 1, 17, 9)[0]
    lib = ndi.correlate(u, np.outer(w, w), mode="constant", cval=0.0)
    assert np.max(np.abs(o.gaussian_apply(u, w) - lib)) < 1e-13


def test_gaussian_matrix_symmetric_bounded_and_indefinite():
    # Assumption 2 holds with M = 1; the truncated kernel is NOT positive
    # semidefinite (the lemma's claim <G u, u> >= 0 fails for the 5x5 taps).
    w = o.gaussian_taps(1.5, 2)
    G = o.assemble_gaussian(24, 24, w).toarray()
    assert np.array_equal(G, G.T)
    ev = np.linalg.eigvalsh(G)
    assert ev.max() <= 1.0 + 1e-12
    # 1-D symbol minimum of the taps bounds the 2-D spectrum from below
    xi = np.linspace(0, np.pi, 20001)
    sym = w[2] + 2 * w[3] * np.cos(xi) + 2 * w[4] * np.cos(2 * xi)
    assert sym.min() < -0.06
    assert ev.min() < 0.0 and ev.min() >= sym.min() * sym.max() - 1e-12


def test_face_gradients_by_hand():
    u = np.arange(1.0, 13.0).reshape(1, 3, 4)      # u(i, j) = 1 + i + 4 j
    gnx, gtx, gny, gty = o.face_gradients(u)
    assert gnx.shape == (1, 3, 5) and gny.shape == (1, 4, 4)
    # interior x-face between (1, 1) and (2, 1): normal 1, tangential (u(1,2)-u(1,0))/2 = 4
    assert gnx[0, 1, 2] == 1.0 and gtx[0, 1, 2] == 4.0
    # left border face: ghost cell has zero tangential difference
    assert gnx[0, 1, 0] == u[0, 1, 0] and gtx[0, 1, 0] == 0.0
    # right border face: normal 0 - u(3, 1), tangential at cell 3
    assert gnx[0, 1, 4] == -u[0, 1, 3] and gtx[0, 1, 4] == (u[0, 2, 3] - u[0, 0, 3]) / 2
    # top border y-face at column 2: normal u(2,0) - 0, tangential at ghost row 0
    assert gny[0, 0, 2] == u[0, 0, 2] and gty[0, 0, 2] == 0.0
    # y-face between rows 0 and 1 at column 0: tangential (u(1,0) - 0)/2
    assert gny[0, 1, 0] == 4.0 and gty[0, 1, 0] == u[0, 0, 1] / 2


def test_diffusivity_literal_values():
    # Section II-B: D = 1 / (|grad u| + eps) with eps = 1e-3 (Section IV-B) and
    # |grad u| the Euclidean norm of (normal, tangential) differences.  Values
    # worked by hand: |(3, 4)| = 5, |(5, 12)| = 13, |(0.6, 0.8)| = 1.  A
    # doubled eps, an l1 norm or a squared norm each miss these.
    gn = np.array([3.0, 5.0, 0.6, 0.0, 1.0, -3.0])
    gt = np.array([4.0, 12.0, 0.8, 0.0, 0.0, -4.0])
    want = np.array([0.19996000799840032, 0.076917160218444735, 0.99900099900099900, 1000.0,
                     0.99900099900099900, 0.19996000799840032])
    D = o.diffusivity(gn, gt, 1e-3)
    assert np.max(np.abs(D - want) / want) <= 4e-16, D
    assert D[3] == 1000.0                                   # flat: D = 1 / eps exactly
    assert np.array_equal(o.diffusivity(gn, gt, 1e-3, edge_preserving=False), np.ones(6))
    # the face coefficients of a field whose face differences are these values
    u = np.zeros((1, 3, 3))
    u[0, 1, 1] = 3.0                  # x-face left of (1, 1): normal 3, tangential (u(0,2) - u(0,0)) / 2
    u[0, 2, 0], u[0, 0, 0] = 8.0, 0.0
    Dx, _ = o.face_coefficients(u)
    assert abs(Dx[0, 1, 1] - 0.19996000799840032) <= 1e-16


def test_diffusivity_assumption_1():
    # D(p) = 1/(|p| + eps) >= nu (1 + |p|)^-1 with nu = 1 since eps <= 1
    s = np.concatenate([np.linspace(0, 10, 1001), np.logspace(-8, 6, 200)])
    D = o.diffusivity(s, np.zeros_like(s), P.eps)
    assert np.all(D >= 1.0 / (1.0 + s))
    assert D.max() <= 1.0 / P.eps


@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (7, 5), (12, 12)])
def test_stencil_matches_assembled_matrix(H, W):
    u = _rand_field(H * 10 + W, 3, H, W)
    v = _rand_field(H * 10 + W + 1, 3, H, W)
    lam = _rand_field(3, 1, H, W, 0.5)[0]
    w = o.gaussian_taps(P.sigma, P.g_radius)
    Dx, Dy = o.face_coefficients(u, P)
    Lv = o.operator_apply(v, Dx, Dy, lam, w, P)
    for c in range(3):
        L = o.assemble_operator(Dx[c], Dy[c], lam, w, P)
        assert np.max(np.abs(L @ v[c].reshape(-1) - Lv[c].reshape(-1))) < 1e-11
        d = o.jacobi_diagonal(Dx, Dy, lam, w, P)[c]
        assert np.max(np.abs(L.diagonal() - d.reshape(-1))) < 1e-11


def test_diffusion_matrix_weak_form_energy():
    # <K v, v> = sum over faces of D (difference across the face)^2, ghost = 0
    H, W = 9, 7
    u = _rand_field(2, 1, H, W)[0]
    v = _rand_field(4, 1, H, W)[0]
    Dx, Dy = o.face_coefficients(u[None], P)
    K = o.assemble_diffusion(Dx[0], Dy[0])
    V = np.pad(v, 1)
    e = np.sum(Dx[0] * (V[1:-1, 1:] - V[1:-1, :-1]) ** 2) + np.sum(Dy[0] * (V[1:, 1:-1] - V[:-1, 1:-1]) ** 2)
    assert abs(v.reshape(-1) @ (K @ v.reshape(-1)) - e) < 1e-9 * e


def test_operator_structure_and_coercivity():
    # Section III: K symmetric positive definite; with constant lambda the
    # whole operator is symmetric; its symmetric part stays positive definite
    # for the lambda range of the method (checked on small grids).
    H, W = 10, 9
    u = _rand_field(8, 1, H, W, 20.0)
    w = o.gaussian_taps(P.sigma, P.g_radius)
    Dx, Dy = o.face_coefficients(u, P)
    K = o.assemble_diffusion(Dx[0], Dy[0]).toarray()
    assert np.array_equal(K, K.T)
    np.linalg.cholesky(K)
    lam_const = np.full((H, W), 0.3)
    Lc = o.assemble_operator(Dx[0], Dy[0], lam_const, w, P).toarray()
    assert np.allclose(Lc, Lc.T, rtol=0, atol=1e-15)
    rng = np.random.default_rng(1)
    lam = P.lambda0 * np.exp(-P.beta_lambda * (1 - rng.uniform(0, 1, size=(H, W))))
    L = o.assemble_operator(Dx[0], Dy[0], lam, w, P).toarray()
    assert not np.allclose(L, L.T)
    assert np.linalg.eigvalsh(0.5 * (L + L.T)).min() > 0


def test_transpose_equivariance_and_mirror_reading():
    # the literal face coefficients are transpose-equivariant but not
    # mirror-equivariant (tangential difference at the lower-index cell)
    H, W = 8, 11
    u = _rand_field(9, 3, H, W)
    phi = _rand_field(10, 3, H, W)
    lam = _rand_field(11, 1, H, W, 0.5)[0]
    r, _ = o.residual(u, phi, lam, P)
    rT, _ = o.residual(u.transpose(0, 2, 1), phi.transpose(0, 2, 1), lam.T, P)
    assert np.max(np.abs(rT - r.transpose(0, 2, 1))) < 1e-12
    rM, _ = o.residual(u[:, :, ::-1], phi[:, :, ::-1], lam[:, ::-1], P)
    assert np.max(np.abs(rM - r[:, :, ::-1])) > 1e-6


def test_channels_are_independent():
    H, W = 6, 7
    u = _rand_field(12, 3, H, W)
    phi = _rand_field(13, 3, H, W)
    lam = _rand_field(14, 1, H, W, 0.5)[0]
    r, _ = o.residual(u, phi, lam, P)
    for c in range(3):
        rc, _ = o.residual(u[c:c + 1], phi[c:c + 1], lam, P)
        assert np.array_equal(rc[0], r[c])


def test_residual_matches_assembled_definition():
    H, W = 9, 8
    u = _rand_field(15, 3, H, W)
    phi = _rand_field(16, 3, H, W)
    lam = _rand_field(17, 1, H, W, 0.5)[0]
    w = o.gaussian_taps(P.sigma, P.g_radius)
    r, rho = o.residual(u, phi, lam, P)
    Dx, Dy = o.face_coefficients(u, P)
    num = 0.0
    for c in range(3):
        L = o.assemble_operator(Dx[c], Dy[c], lam, w, P)
        rc = phi[c].reshape(-1) - L @ u[c].reshape(-1)
        assert np.max(np.abs(rc - r[c].reshape(-1))) < 1e-11
        num += rc @ rc
    assert abs(rho - np.sqrt(num) / np.linalg.norm(phi)) < 1e-14


def test_ablation_switches():
    H, W = 6, 6
    u = _rand_field(18, 1, H, W)
    lam = _rand_field(19, 1, H, W, 0.5)[0]
    w = o.gaussian_taps(P.sigma, P.g_radius)
    q = o.with_params(edge_preserving=False)
    Dx, Dy = o.face_coefficients(u, q)
    assert np.all(Dx == 1.0) and np.all(Dy == 1.0)
    q2 = o.with_params(nonlocal_term=False)
    Dx, Dy = o.face_coefficients(u, q2)
    assert np.array_equal(o.operator_apply(u, Dx, Dy, lam, w, q2), -o.divergence(u, Dx, Dy))


@pytest.mark.parametrize("lam0", [0.05, 0.4])
def test_analytic_start_solves_smooth_interior(lam0):
    # Where Phi is linear and lambda constant, B = Phi / lambda is linear too:
    # the normalised symmetric Gaussian reproduces it and the constant-slope
    # flux has zero divergence, so the residual of B vanishes on every pixel
    # more than R + 1 from the zero boundary.  A wrong base (Phi lambda,
    # Phi / (lambda w0^2), Phi) leaves a residual there.
    H, W = 24, 30
    R = o.DEFAULT.g_radius
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    phi = np.stack([0.3 + 0.01 * xx + 0.02 * yy, 0.5 - 0.015 * yy, 0.2 + 0.005 * xx])
    lam = np.full((H, W), lam0)
    B = o.analytic_start(phi, lam)
    r, _ = o.residual(B, phi, lam)
    inner = r[:, R + 2:H - R - 2, R + 2:W - R - 2]
    assert np.max(np.abs(inner)) <= 1e-11 * np.max(np.abs(phi / lam0))
    for wrong in (phi * lam0, phi / (lam0 * o.gaussian_taps(o.DEFAULT.sigma, R)[R] ** 2), phi):
        rw, _ = o.residual(wrong, phi, lam)
        assert np.max(np.abs(rw[:, R + 2:H - R - 2, R + 2:W - R - 2])) > 1e-3
    # without the nonlocal term, or where lambda = 0, the base is Phi itself
    q = o.with_params(nonlocal_term=False)
    assert np.array_equal(o.analytic_start(phi, lam, q), phi)
    lz = lam.copy()
    lz[3, 4] = 0.0
    Bz = o.analytic_start(phi, lz)
    assert np.array_equal(Bz[:, 3, 4], phi[:, 3, 4])
