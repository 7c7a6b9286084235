"""The allocation-free residual entry point against the workspace one.

dehaze_residual_noalloc runs the same residual kernels as dehaze_residual
with its partial sums in a library-owned device array instead of a caller
workspace, and writes rho to device memory.  Both calls are made through the
C ABI on the same device inputs; r must agree bit for bit (same kernels, same
order) and rho to a few float64 ulps (the same two sums, correctly rounded
square roots and one division on the device versus on the host).  Two calls
in a row, the second on a smaller image, check that the array keeps nothing
from the previous call that matters.  The oracle pins the value itself.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import ctx, dev, host, require_gpu, say
from oracle import dehaze_ref as o

pytestmark = pytest.mark.gpu


def _case(H, W, seed):
    img = synth.hazy_image(H, W, seed, beta_haze=(0.5, 2.0), occlusion=True)
    pr = o.prior(img["I"])
    t32 = pr["t"].astype(np.float32)
    A32 = pr["A"].astype(np.float32)
    lam = o.adaptive_weight(t32.astype(np.float64)).astype(np.float32)
    phi = o.reconstruction(img["I"], t32, A32, o.DEFAULT.t0).astype(np.float32)
    rng = np.random.default_rng(seed)
    u = (phi + rng.uniform(-1, 1, size=phi.shape)).astype(np.float32)
    return u, phi, lam


def _compare(d, H, W, seed):
    u, phi, lam = _case(H, W, seed)
    du, dphi, dlam = dev(u), dev(phi), dev(lam)
    say(f"noalloc residual H={H} W={W} seed={seed}")
    rho_ws, r_ws = d.dehaze_residual(ctx(), du, dphi, dlam, want_r=True)
    rho_dev = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    r_na = torch.full_like(du, float("nan"))
    d.dehaze_residual_noalloc(ctx(), du, dphi, dlam, rho_dev, r=r_na)
    rho_na = float(host(rho_dev)[0])
    assert np.array_equal(host(r_na), host(r_ws))
    assert abs(rho_na - rho_ws) <= 4 * np.spacing(rho_ws), (rho_na, rho_ws)
    # and both agree with the oracle's residual of the same float32 u
    _, rho_ref = o.residual(u.astype(np.float64), phi.astype(np.float64), lam.astype(np.float64))
    assert abs(rho_na - rho_ref) <= 1e-5 * rho_ref + 4e-6
    # without r the value is the same
    rho2 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    d.dehaze_residual_noalloc(ctx(), du, dphi, dlam, rho2)
    assert float(host(rho2)[0]) == rho_na


def test_noalloc_residual_matches_workspace_entry_point():
    require_gpu()
    import paper_2506_08793_amd as d
    # larger first, then smaller: stale partial sums past the second image's
    # block count must not reach its result
    _compare(d, 300, 517, 61)
    _compare(d, 37, 70, 62)


def test_noalloc_residual_rejects_oversized_images():
    require_gpu()
    import paper_2506_08793_amd as d
    # ceil(W/64) * ceil(H/16) above the array's block count is refused before
    # any launch; the tensors are never read, so tiny ones stand in
    small = torch.zeros((3, 1, 1), dtype=torch.float32, device="cuda")
    lam = torch.zeros((1, 1), dtype=torch.float32, device="cuda")
    rho = torch.zeros((1,), dtype=torch.float64, device="cuda")
    lib = d.binding.lib()
    import ctypes
    p = d.dehaze_params_default()
    H, W = 8192 + 16, 8192
    rc = lib.dehaze_residual_noalloc(ctx().handle, small.data_ptr(), small.data_ptr(), lam.data_ptr(), H, W,
                                     ctypes.byref(p), None, rho.data_ptr(), None)
    assert rc == d.binding.EINVAL
    assert b"allocation-free scratch holds" in lib.dehaze_last_error()
