"""FP64 CPU oracle for the PDE dehazing method (test infrastructure only).

This module is a plain, slow, obviously correct statement of what the method
computes.  It exists to check the GPU path; nothing in the product package may
import or call it (only the tests, the smoke check and the CPU baseline leg of
the benchmark do).  It shares no code with the HIP kernels.

Arithmetic is float64 throughout.  Inputs are the same float32 arrays the GPU
receives, promoted exactly to float64.  Arrays are planar: colour images are
(3, H, W), scalar fields (H, W); x is the column index i, y the row index j.

Paper sections followed:
  * Section II-A: scattering model, reconstruction operator Phi, threshold t0.
  * Section II-B: diffusivity D = (|grad u| + eps)^-1.
  * Section II-C: Gaussian operator G (integral over the image domain).
  * Section II-D: dark channel, transmission t = 1 - omega t_d, weight lambda(t).
  * Eq. (main PDE): -div(D(grad u) grad u) + lambda(t) G(u) = Phi.
  * Section III: weak form, coercivity (checked on the assembled operator).
  * Appendix A-1: relaxed fixed-point update and its step bound.
  * Appendix A-2: face-centred discretisation of the diffusion term, the 5x5
    Gaussian kernel.

Readings taken where the paper is silent or ambiguous (all are parameters):
  * A is estimated with the dark-channel-prior rule: the top HW/1000 pixels of
    the dark channel (ties to the lower linear index), then the brightest of
    them by R+G+B (float64 sum, ties to the lower index).
  * t0 = 0.1; t is clamped to [0, 1]; sigma = 1.5 (the paper uses 2.0, kept as
    a parameter); the 5x5 taps are normalised to sum 1; G and u are extended
    by zero outside the image (H0^1 boundary); channels are solved
    independently, sharing t and lambda.
  * Face coefficients use the forward normal difference and the central
    tangential difference at the lower-index cell, exactly as Appendix A-2
    writes them.
  * lambda follows the printed formula lambda0 exp(-beta (1 - t)).
  * The guided filter and the multiscale dark channel that Table II ablates
    are not defined in the paper; their readings (He, Sun and Tang's guided
    filter with the channel-mean guide; t_d averaged over patch sides patch,
    patch/2, ...) are off by default and parity unpinned against the paper:
    their tests pin them to brute force and closed forms only.
  * The warm start begins from B = Phi / lambda, the solution of lambda u =
    Phi to which the main PDE reduces where u is smooth (analytic_start).
  * Three iterations share the fixed point r(u) = 0: the paper's explicit
    relaxed update, a diagonally scaled (Jacobi) form of it, and the
    lagged-diffusivity (Picard) iteration u_{n+1} = L(D(u_n))^-1 Phi.
  * Outer acceleration of the lagged-diffusivity iteration (not in the
    paper, which leaves the iteration count open): nonlinear GMRES in the
    sense of Washio and Oosterlee, with the Picard step as its
    preconditioner (ngmres_solve).  It has the same fixed point.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.lib.stride_tricks import sliding_window_view


@dataclass(frozen=True)
class Params:
    """Method parameters (Section IV-B values, sigma from the workloads)."""
    patch: int = 15           # dark-channel patch side (Section II-D)
    omega: float = 0.95       # transmission factor (Section II-D)
    t0: float = 0.1           # reconstruction threshold (Section II-A, value is a reading)
    eps: float = 1e-3         # diffusivity stabiliser (Section II-B)
    sigma: float = 1.5        # Gaussian width (Section II-C uses 2.0)
    g_radius: int = 2         # 5x5 kernel (Appendix A-2)
    lambda0: float = 0.5      # Section II-D
    beta_lambda: float = 3.0  # Section II-D (sharpness of lambda, not haze density)
    tau: float = 0.2          # Appendix A-1 relaxation
    theta: float = 0.8        # damping of the diagonally scaled update
    atm_divisor: int = 1000   # top HW/atm_divisor dark-channel pixels feed A
    # Ablation switches (Table II rows with a definition in the paper).
    nonlocal_term: bool = True
    adaptive: bool = True
    edge_preserving: bool = True
    # Table II also ablates a guided filter and a multiscale dark channel,
    # which the paper never defines.  Readings (off by default, so the
    # printed formulation is the default): the guided filter of He, Sun and
    # Tang refines t with the channel mean of I as guide; the multiscale dark
    # channel averages t_d over the patch sides patch, patch/2, patch/4, ...
    guided_radius: int = 0    # 0: no refinement
    guided_eps: float = 1e-3
    dark_scales: int = 1      # number of patch sides averaged


DEFAULT = Params()


# ------------------------------------------------------------------ front end
def unit_from_u8(codes: np.ndarray) -> np.ndarray:
    """8-bit code -> float32 intensity code/255, correctly rounded.

    The float64 quotient of two small integers rounded once more to float32
    equals the correctly rounded float32 quotient (53 >= 2*24 + 2).
    """
    return (np.asarray(codes, dtype=np.float64) / 255.0).astype(np.float32)


def patch_min(I: np.ndarray, patch: int) -> np.ndarray:
    """Per-channel minimum over the patch centred at each pixel (Section II-D).

    The window is clipped to the image (equivalently: +inf outside).  The
    result holds exact copies of input values, returned as float64.
    """
    if patch < 1 or patch % 2 == 0:
        raise ValueError("patch must be odd and positive")
    I = np.asarray(I, dtype=np.float64)
    r = patch // 2
    C, H, W = I.shape
    P = np.full((C, H + 2 * r, W + 2 * r), np.inf)
    P[:, r:r + H, r:r + W] = I
    win = sliding_window_view(P, (patch, patch), axis=(1, 2))
    return win.min(axis=(-2, -1))


def dark_channel(m: np.ndarray) -> np.ndarray:
    """Raw dark channel: minimum over colour channels of the patch minima."""
    return np.min(m, axis=0)


def atmospheric_light(I: np.ndarray, dc: np.ndarray, atm_divisor: int = 1000):
    """Dark-channel-prior estimate of A (the paper takes A as given).

    k = max(1, floor(H W / atm_divisor)) pixels with the largest dark channel
    (ties: lower linear index j*W + i); among them the pixel with the largest
    R+G+B, summed in float64 as (R+G)+B (ties: lower index).  Returns
    (A as float64 copies of the input values, linear index of that pixel).
    """
    I = np.asarray(I, dtype=np.float64)
    C, H, W = I.shape
    n = H * W
    k = max(1, n // int(atm_divisor))
    flat = dc.reshape(-1)
    idx = np.arange(n)
    order = np.lexsort((idx, -flat))          # dark channel descending, index ascending
    cand = order[:k]
    Iflat = I.reshape(C, -1)
    s = (Iflat[0, cand] + Iflat[1, cand]) + Iflat[2, cand]
    best = cand[np.lexsort((cand, -s))[0]]
    return Iflat[:, best].copy(), int(best)


def transmission(m: np.ndarray, A, omega: float):
    """t_d = min_c min_patch I^c / A^c and t = clamp(1 - omega t_d, 0, 1).

    The patch minimum is taken before the division, which is monotone for
    A^c > 0 and so commutes with it.
    """
    A = np.asarray(A, dtype=np.float64)
    if np.any(A <= 0):
        raise ValueError("atmospheric light must be positive")
    td = np.min(m / A[:, None, None], axis=0)
    t = np.clip(1.0 - omega * td, 0.0, 1.0)
    return td, t


def scale_patches(patch: int, scales: int) -> list:
    """Patch sides of the multiscale dark channel: ((patch - 1) >> k) | 1."""
    return [((patch - 1) >> k) | 1 for k in range(scales)]


def multiscale_transmission(I: np.ndarray, A, p: Params):
    """t_d averaged over the patch sides of scale_patches (a reading of the
    multiscale dark channel Table II names) and t = clamp(1 - omega t_d, 0, 1)."""
    A = np.asarray(A, dtype=np.float64)
    tds = []
    for side in scale_patches(p.patch, p.dark_scales):
        td_k, _ = transmission(patch_min(I, side), A, p.omega)
        tds.append(td_k)
    td = np.mean(tds, axis=0)
    return td, np.clip(1.0 - p.omega * td, 0.0, 1.0)


def box_mean(x: np.ndarray, r: int) -> np.ndarray:
    """Mean of x over the (2r+1) x (2r+1) window centred at each pixel,
    clipped to the image (the guided filter's mean; He, Sun and Tang)."""
    x = np.asarray(x, dtype=np.float64)
    H, W = x.shape
    c = np.zeros((H + 1, W + 1))
    c[1:, 1:] = np.cumsum(np.cumsum(x, axis=0), axis=1)
    ys = np.arange(H)
    xs = np.arange(W)
    y0, y1 = np.maximum(ys - r, 0), np.minimum(ys + r, H - 1) + 1
    x0, x1 = np.maximum(xs - r, 0), np.minimum(xs + r, W - 1) + 1
    s = (c[y1][:, x1] - c[y0][:, x1]) - (c[y1][:, x0] - c[y0][:, x0])
    n = np.outer(y1 - y0, x1 - x0)
    return s / n


def guided_filter(G: np.ndarray, q_in: np.ndarray, r: int, eps: float) -> np.ndarray:
    """Guided filter (He, Sun and Tang): in every window the output is a linear
    function a G + b of the guide, a = cov(G, q) / (var(G) + eps) and
    b = mean(q) - a mean(G); each pixel averages the a, b of the windows
    covering it: out = mean(a) G + mean(b)."""
    G = np.asarray(G, dtype=np.float64)
    q_in = np.asarray(q_in, dtype=np.float64)
    mG, mq = box_mean(G, r), box_mean(q_in, r)
    cov = box_mean(G * q_in, r) - mG * mq
    var = box_mean(G * G, r) - mG * mG
    a = cov / (var + eps)
    b = mq - a * mG
    return box_mean(a, r) * G + box_mean(b, r)


def refine_transmission(I: np.ndarray, t: np.ndarray, p: Params) -> np.ndarray:
    """Guided-filter refinement of t (a reading of the guided filter Table II
    names): guide = channel mean of I, input = t as stored (float32), output
    clamped to [0, 1]."""
    I = np.asarray(I, dtype=np.float64)
    guide = ((I[0] + I[1]) + I[2]) / 3.0
    t32 = np.asarray(t, dtype=np.float32).astype(np.float64)
    return np.clip(guided_filter(guide, t32, p.guided_radius, p.guided_eps), 0.0, 1.0)


def adaptive_weight(t: np.ndarray, p: Params = DEFAULT) -> np.ndarray:
    """lambda(t) = lambda0 exp(-beta (1 - t)) (Section II-D); lambda0 when not adaptive."""
    t = np.asarray(t, dtype=np.float64)
    if not p.adaptive:
        return np.full_like(t, p.lambda0)
    return p.lambda0 * np.exp(-p.beta_lambda * (1.0 - t))


def reconstruction(I: np.ndarray, t: np.ndarray, A, t0: float) -> np.ndarray:
    """Phi(I, t, A) = (I - A (1 - t)) / max(t, t0) per channel (Section II-A)."""
    I = np.asarray(I, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    return (I - A[:, None, None] * (1.0 - t[None])) / np.maximum(t, t0)[None]


def analytic_start(phi: np.ndarray, lam: np.ndarray, p: Params = DEFAULT) -> np.ndarray:
    """B = Phi / lambda: where u is smooth, G(u) = u and the diffusion term of
    the main PDE vanishes, leaving lambda u = Phi.  Without the nonlocal term
    (or where lambda = 0) B = Phi.  A starting iterate, not part of the
    method; the warm start of the solve (a reading, Section I's closing
    remark on hybrids)."""
    phi = np.asarray(phi, dtype=np.float64)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), phi.shape[-2:])
    if not p.nonlocal_term:
        return phi.copy()
    safe = np.where(lam > 0, lam, 1.0)
    return np.where(lam[None] > 0, phi / safe[None], phi)


def prior(I: np.ndarray, p: Params = DEFAULT, A=None) -> dict:
    """The whole front end: patch minima, dark channel, A, t_d, t, lambda, Phi."""
    m = patch_min(I, p.patch)
    dc = dark_channel(m)
    if A is None:
        A, a_idx = atmospheric_light(I, dc, p.atm_divisor)
    else:
        A, a_idx = np.asarray(A, dtype=np.float64), -1
    if p.dark_scales > 1:
        td, t = multiscale_transmission(I, A, p)
    else:
        td, t = transmission(m, A, p.omega)
    t_raw = t
    if p.guided_radius > 0:
        t = refine_transmission(I, t, p)
    lam = adaptive_weight(t, p)
    phi = reconstruction(I, t, A, p.t0)
    return {"m": m, "dc": dc, "A": A, "A_index": a_idx, "t_d": td, "t_raw": t_raw, "t": t,
            "lam": lam, "phi": phi}


# ------------------------------------------------------------------ operators
def gaussian_taps(sigma: float, radius: int) -> np.ndarray:
    """1-D taps w_a proportional to exp(-a^2 / 2 sigma^2), a = -R..R, summing to 1.

    The 2-D kernel of Section II-C factors as w_a w_b; truncating it to the
    (2R+1)^2 window of Appendix A-2 and normalising the taps is the reading.
    """
    a = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(a * a) / (2.0 * sigma * sigma))
    return g / g.sum()


def gaussian_apply(u: np.ndarray, w: np.ndarray) -> np.ndarray:
    """G(u)(i, j) = sum_{a,b} w_a w_b u(i+a, j+b), u extended by zero (Section II-C)."""
    u = np.asarray(u, dtype=np.float64)
    R = (len(w) - 1) // 2
    H, W = u.shape[-2:]
    pad = [(0, 0)] * (u.ndim - 2) + [(R, R), (R, R)]
    P = np.pad(u, pad)
    out = np.zeros_like(u)
    for b in range(-R, R + 1):          # row offset
        for a in range(-R, R + 1):      # column offset
            out += w[a + R] * w[b + R] * P[..., R + b:R + b + H, R + a:R + a + W]
    return out


def face_gradients(u: np.ndarray):
    """Normal and tangential differences on every x-face and y-face (Appendix A-2).

    x-face f (0..W) sits between cells i = f-1 and i+1 = f of a row; its normal
    difference is u(i+1, j) - u(i, j) and its tangential difference
    (u(i, j+1) - u(i, j-1)) / 2 is taken at the lower-index cell i.  y-faces are
    the same with rows and columns swapped.  u is zero outside the image.
    Shapes: x-faces (..., H, W+1), y-faces (..., H+1, W).
    """
    u = np.asarray(u, dtype=np.float64)
    H, W = u.shape[-2:]
    pad = [(0, 0)] * (u.ndim - 2) + [(1, 1), (1, 1)]
    U = np.pad(u, pad)                  # U[j+1, i+1] = u(i, j)
    gnx = U[..., 1:H + 1, 1:W + 2] - U[..., 1:H + 1, 0:W + 1]
    gtx = (U[..., 2:H + 2, 0:W + 1] - U[..., 0:H, 0:W + 1]) / 2.0
    gny = U[..., 1:H + 2, 1:W + 1] - U[..., 0:H + 1, 1:W + 1]
    gty = (U[..., 0:H + 1, 2:W + 2] - U[..., 0:H + 1, 0:W]) / 2.0
    return gnx, gtx, gny, gty


def diffusivity(gn: np.ndarray, gt: np.ndarray, eps: float, edge_preserving: bool = True):
    """D = 1 / (|(gn, gt)| + eps) (Section II-B); 1 when edge preservation is off."""
    if not edge_preserving:
        return np.ones_like(gn)
    return 1.0 / (np.sqrt(gn * gn + gt * gt) + eps)


def face_coefficients(u: np.ndarray, p: Params = DEFAULT):
    """Frozen face coefficients (Dx, Dy) at the iterate u."""
    gnx, gtx, gny, gty = face_gradients(u)
    return (diffusivity(gnx, gtx, p.eps, p.edge_preserving),
            diffusivity(gny, gty, p.eps, p.edge_preserving))


def divergence(u: np.ndarray, Dx: np.ndarray, Dy: np.ndarray) -> np.ndarray:
    """div(D grad u) with face fluxes D * (normal difference) (Appendix A-2)."""
    gnx, _, gny, _ = face_gradients(u)
    qx = Dx * gnx
    qy = Dy * gny
    return (qx[..., :, 1:] - qx[..., :, :-1]) + (qy[..., 1:, :] - qy[..., :-1, :])


def effective_lambda(lam: np.ndarray, p: Params) -> np.ndarray:
    return np.zeros_like(lam) if not p.nonlocal_term else lam


def operator_apply(v: np.ndarray, Dx, Dy, lam, w, p: Params = DEFAULT) -> np.ndarray:
    """L_D v = -div(D grad v) + lambda G(v) with D frozen (eq. main PDE)."""
    lam_e = effective_lambda(np.asarray(lam, dtype=np.float64), p)
    return -divergence(v, Dx, Dy) + lam_e * gaussian_apply(v, w)


def residual(u: np.ndarray, phi: np.ndarray, lam: np.ndarray, p: Params = DEFAULT):
    """r(u) = Phi - L_{D(u)} u and rho = ||r||_2 / ||Phi||_2 over all channels."""
    w = gaussian_taps(p.sigma, p.g_radius)
    Dx, Dy = face_coefficients(u, p)
    r = np.asarray(phi, dtype=np.float64) - operator_apply(u, Dx, Dy, lam, w, p)
    nphi = np.sqrt(np.sum(np.asarray(phi, dtype=np.float64) ** 2))
    rho = np.sqrt(np.sum(r * r)) / nphi if nphi > 0 else np.sqrt(np.sum(r * r))
    return r, float(rho)


def jacobi_diagonal(Dx, Dy, lam, w, p: Params = DEFAULT) -> np.ndarray:
    """Diagonal of the frozen operator: sum of the four face D plus lambda w0^2."""
    R = (len(w) - 1) // 2
    lam_e = effective_lambda(np.asarray(lam, dtype=np.float64), p)
    return (Dx[..., :, :-1] + Dx[..., :, 1:] + Dy[..., :-1, :] + Dy[..., 1:, :]
            + lam_e * (w[R] * w[R]))


# --------------------------------------------------------------- assembly
def assemble_diffusion(Dx: np.ndarray, Dy: np.ndarray) -> sp.csr_matrix:
    """Matrix of -div(D grad .) for one channel; unknown (i, j) has index j*W + i.

    Written face by face, independently of the stencil code above: an interior
    face with coefficient D couples its two cells by [[D, -D], [-D, D]]; a face
    on the image border touches one cell and a zero ghost, adding D to its
    diagonal.
    """
    H, W = Dx.shape[0], Dy.shape[1]
    n = H * W
    rows, cols, vals = [], [], []
    # x-faces: face f of row j lies between cells lo = f-1 and hi = f.
    jj, ff = np.meshgrid(np.arange(H), np.arange(W + 1), indexing="ij")
    # y-faces: face f of column i lies between rows lo = f-1 and hi = f.
    gg, ii = np.meshgrid(np.arange(H + 1), np.arange(W), indexing="ij")
    for D, lo, hi, ok_lo, ok_hi in (
            (Dx, jj * W + (ff - 1), jj * W + ff, ff - 1 >= 0, ff < W),
            (Dy, (gg - 1) * W + ii, gg * W + ii, gg - 1 >= 0, gg < H)):
        D, lo, hi, ok_lo, ok_hi = (a.reshape(-1) for a in (D, lo, hi, ok_lo, ok_hi))
        both = ok_lo & ok_hi
        for sel, a, b, sign in ((ok_lo, lo, lo, 1.0), (ok_hi, hi, hi, 1.0),
                                (both, lo, hi, -1.0), (both, hi, lo, -1.0)):
            rows.append(a[sel]); cols.append(b[sel]); vals.append(sign * D[sel])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


_G_CACHE: dict = {}


def assemble_gaussian(H: int, W: int, w: np.ndarray) -> sp.csr_matrix:
    """Matrix of G on an H x W grid with zero extension: G[p, q] = w_a w_b."""
    key = (H, W, tuple(np.asarray(w).tolist()))
    if key in _G_CACHE:
        return _G_CACHE[key]
    R = (len(w) - 1) // 2
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    jj, ii = jj.reshape(-1), ii.reshape(-1)
    rows, cols, vals = [], [], []
    for b in range(-R, R + 1):
        for a in range(-R, R + 1):
            ok = (jj + b >= 0) & (jj + b < H) & (ii + a >= 0) & (ii + a < W)
            rows.append((jj * W + ii)[ok]); cols.append(((jj + b) * W + ii + a)[ok])
            vals.append(np.full(int(ok.sum()), w[a + R] * w[b + R]))
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(H * W, H * W))
    if len(_G_CACHE) > 8:
        _G_CACHE.clear()
    _G_CACHE[key] = G
    return G


def assemble_operator(Dx, Dy, lam, w, p: Params = DEFAULT) -> sp.csr_matrix:
    """L = K(D) + diag(lambda) G for one channel."""
    H, W = lam.shape
    K = assemble_diffusion(Dx, Dy)
    lam_e = effective_lambda(np.asarray(lam, dtype=np.float64), p)
    G = assemble_gaussian(H, W, w)
    return (K + sp.diags(lam_e.reshape(-1)) @ G).tocsr()


# ------------------------------------------------------------------ schemes
def explicit_step(u, phi, lam, p: Params = DEFAULT):
    """Appendix A-1: u + tau [div(D_n grad u) - lambda G(u) + Phi], D_n = D(u)."""
    r, _ = residual(u, phi, lam, p)
    return np.asarray(u, dtype=np.float64) + p.tau * r


def jacobi_sweep(u, phi, lam, p: Params = DEFAULT):
    """Diagonally scaled form of the same update: u + theta r(u) / d(u)."""
    w = gaussian_taps(p.sigma, p.g_radius)
    u = np.asarray(u, dtype=np.float64)
    Dx, Dy = face_coefficients(u, p)
    r = np.asarray(phi, dtype=np.float64) - operator_apply(u, Dx, Dy, lam, w, p)
    d = jacobi_diagonal(Dx, Dy, lam, w, p)
    return u + p.theta * r / d


def picard_step(u, phi, lam, p: Params = DEFAULT):
    """Lagged diffusivity: freeze D_n = D(u_n) and solve L(D_n) u_{n+1} = Phi per channel."""
    w = gaussian_taps(p.sigma, p.g_radius)
    u = np.asarray(u, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    Dx, Dy = face_coefficients(u, p)
    out = np.empty_like(u)
    for c in range(u.shape[0]):
        L = assemble_operator(Dx[c], Dy[c], lam, w, p).tocsc()
        # Sparse LU with a minimum-degree ordering of the symmetric pattern.
        lu = spla.splu(L, permc_spec="MMD_AT_PLUS_A")
        out[c] = lu.solve(phi[c].reshape(-1)).reshape(u.shape[1:])
    return out


def explicit_step_bound(p: Params = DEFAULT, M: float = 1.0) -> float:
    """Appendix A-1 step bound 2 / (||D Laplacian|| + lambda M) at its worst case.

    D <= 1/eps and the 5-point Laplacian has norm <= 8, lambda <= lambda0.
    """
    return 2.0 / (8.0 / p.eps + p.lambda0 * M)


@dataclass
class SolveResult:
    u: np.ndarray
    rho: list = field(default_factory=list)   # rho before each step, then the final one
    steps: int = 0


def solve(phi, lam, scheme: str, p: Params = DEFAULT, steps: int = None,
          rel_tol: float = None, u0=None, max_steps: int = 100000) -> SolveResult:
    """Run one of 'explicit', 'jacobi', 'picard' from u0 (default Phi).

    Stops after ``steps`` updates, or when rho <= rel_tol (checked before each
    update), whichever is given.
    """
    step = {"explicit": explicit_step, "jacobi": jacobi_sweep, "picard": picard_step}[scheme]
    u = np.array(phi if u0 is None else u0, dtype=np.float64)
    res = SolveResult(u=u)
    n = 0
    limit = steps if steps is not None else max_steps
    while True:
        _, rho = residual(u, phi, lam, p)
        res.rho.append(rho)
        if (rel_tol is not None and rho <= rel_tol) or n >= limit:
            break
        u = step(u, phi, lam, p)
        n += 1
    res.u, res.steps = u, n
    return res


def ngmres_mix(ut, rt, U, R, reg: float = 1e-10):
    """Least-squares mixing of a trial iterate with earlier ones.

    Given the trial iterate ut with its residual rt and earlier trial iterates
    U[j] with residuals R[j], the coefficients b minimise
    || rt + sum_j b_j (rt - R[j]) ||_2 (over all channels and pixels); they
    solve the normal equations with a Tikhonov shift of reg * trace / n on
    the diagonal, which only matters when the differences are nearly
    dependent.  Returns (u_mix, r_mix, b): the mixed iterate
    ut + sum_j b_j (ut - U[j]) and the same combination of the residuals (the
    residual of u_mix to first order).
    """
    n = len(U)
    if n == 0:
        return np.array(ut, dtype=np.float64), np.array(rt, dtype=np.float64), np.zeros(0)
    ut = np.asarray(ut, dtype=np.float64)
    rt = np.asarray(rt, dtype=np.float64)
    A = np.stack([(rt - np.asarray(Rj, dtype=np.float64)).reshape(-1) for Rj in R], axis=1)
    G = A.T @ A
    h = A.T @ rt.reshape(-1)
    G = G + reg * np.trace(G) / n * np.eye(n)
    b = np.linalg.solve(G, -h)
    u_mix = ut + sum(bj * (ut - np.asarray(Uj, dtype=np.float64)) for bj, Uj in zip(b, U))
    r_mix = rt + sum(bj * (rt - np.asarray(Rj, dtype=np.float64)) for bj, Rj in zip(b, R))
    return u_mix, r_mix, b


def ngmres_solve(phi, lam, p: Params = DEFAULT, depth: int = 5, steps: int = None, rel_tol: float = None,
                 u0=None, max_steps: int = 100000, growth: float = 2.0) -> SolveResult:
    """Lagged-diffusivity iteration accelerated by nonlinear GMRES.

    Step n starts from the trial iterate ut_n and its residual r(ut_n):
      1. mix ut_n with the last `depth` trial iterates (ngmres_mix), giving
         u_mix and the combined residual r_mix;
      2. take the lagged-diffusivity correction from u_mix with D frozen at
         ut_n: ut_{n+1} = u_mix + L(D(ut_n))^-1 r_mix (exact sparse LU);
      3. evaluate r(ut_{n+1}); if rho grows beyond `growth` times the lowest
         rho so far, the history is dropped (the next step is a plain one).
    With depth = 0 this is the lagged-diffusivity iteration itself:
    ut + L(D(ut))^-1 (Phi - L(D(ut)) ut) = L(D(ut))^-1 Phi.  rho is recorded
    for every trial iterate; the result is the last one.
    """
    w = gaussian_taps(p.sigma, p.g_radius)
    phi = np.asarray(phi, dtype=np.float64)
    ut = np.array(phi if u0 is None else u0, dtype=np.float64)
    r, rho = residual(ut, phi, lam, p)
    res = SolveResult(u=ut, rho=[rho])
    U, R = [], []
    best = rho
    n = 0
    limit = steps if steps is not None else max_steps
    while not ((rel_tol is not None and rho <= rel_tol) or n >= limit):
        u_mix, r_mix, _ = ngmres_mix(ut, r, U, R)
        if depth > 0:
            U.append(ut.copy())
            R.append(r.copy())
            if len(U) > depth:
                U.pop(0)
                R.pop(0)
        Dx, Dy = face_coefficients(ut, p)
        delta = np.empty_like(ut)
        for c in range(ut.shape[0]):
            L = assemble_operator(Dx[c], Dy[c], lam, w, p).tocsc()
            delta[c] = spla.splu(L, permc_spec="MMD_AT_PLUS_A").solve(r_mix[c].reshape(-1)).reshape(ut.shape[1:])
        ut = u_mix + delta
        r, rho = residual(ut, phi, lam, p)
        res.rho.append(rho)
        n += 1
        if rho > growth * best:
            U, R = [], []
        best = min(best, rho)
    res.u, res.steps = ut, n
    return res


def dehaze(I: np.ndarray, scheme: str = "picard", p: Params = DEFAULT, steps: int = None,
           rel_tol: float = None, A=None, t=None, u0=None) -> dict:
    """Front end followed by the solve; t and A may be supplied by the caller."""
    if t is None:
        pr = prior(I, p, A=A)
    else:
        A = np.asarray(A, dtype=np.float64)
        t64 = np.asarray(t, dtype=np.float64)
        pr = {"A": A, "t": t64, "lam": adaptive_weight(t64, p),
              "phi": reconstruction(I, t64, A, p.t0)}
    sol = solve(pr["phi"], pr["lam"], scheme, p, steps=steps, rel_tol=rel_tol, u0=u0)
    return {**pr, "u": sol.u, "rho": sol.rho, "steps": sol.steps}


def with_params(**kw) -> Params:
    return replace(DEFAULT, **kw)
