"""Failure detection through the C ABI: non-finite input or a non-positive
airlight is reported as DEHAZE_ENONFINITE (per image in a batch), and the
other images of a batch are unaffected.  Every kernel still runs to its
normal end: the NaN only travels through the arithmetic."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import ctx, dev, host, require_gpu, say
from oracle import dehaze_ref as o

pytestmark = pytest.mark.gpu

ENONFINITE = -5


def _clean(H, W, seed):
    img = synth.hazy_image(H, W, seed, beta_haze=(0.5, 2.0), occlusion=True)
    pr = o.prior(img["I"])
    return img["I"], pr["t"].astype(np.float32), pr["A"].astype(np.float32)


def _nan_image(I, y, x, c=1):
    J = I.copy()
    J[c, y, x] = np.nan
    return J


@pytest.mark.parametrize("scheme", [1, 2])
def test_nan_in_input_solve(scheme):
    require_gpu()
    import paper_2506_08793_amd as d
    I, t, A = _clean(24, 40, 71)
    J = _nan_image(I, 11, 17)
    say(f"nan input, dehaze_solve scheme {scheme}")
    p = d.dehaze_params_default(scheme=scheme, max_outer=200, rel_tol=1e-5)
    with pytest.raises(d.DehazeError) as e:
        d.dehaze_solve(ctx(), dev(J), dev(t), dev(A), params=p)
    assert e.value.code == ENONFINITE
    # the clean image with the same arguments is fine
    u, st = d.dehaze_solve(ctx(), dev(I), dev(t), dev(A), params=p.replace(max_outer=5, rel_tol=0.0))
    assert st["status"] == 0 and np.isfinite(host(u)).all()


@pytest.mark.parametrize("estimate", [False, True])
def test_nan_in_input_batch_flags_only_that_image(estimate):
    require_gpu()
    import paper_2506_08793_amd as d
    cases = [_clean(32, 48, 72), _clean(20, 70, 73), _clean(40, 33, 74)]
    imgs = [dev(c[0]) for c in cases]
    imgs[1] = dev(_nan_image(cases[1][0], 5, 9, c=2))
    t = None if estimate else [dev(c[1]) for c in cases]
    A = None if estimate else [dev(c[2]) for c in cases]
    p = d.dehaze_params_default(max_outer=3000)
    say(f"nan input, dehaze_batch estimate={estimate}")
    us, st, _, _ = d.dehaze_batch(ctx(), imgs, params=p, t=t, A=A, allow_nonfinite=True)
    assert [s["status"] for s in st] == [0, ENONFINITE, 0]
    assert st[0]["converged"] and st[2]["converged"] and not st[1]["converged"]
    with pytest.raises(d.DehazeError) as e:
        d.dehaze_batch(ctx(), imgs, params=p, t=t, A=A)
    assert e.value.code == ENONFINITE
    # images of a batch progress independently: the clean ones equal their
    # solves without the poisoned neighbour
    alone, st2, _, _ = d.dehaze_batch(ctx(), [imgs[0], imgs[2]], params=p,
                                      t=None if t is None else [t[0], t[2]],
                                      A=None if A is None else [A[0], A[2]])
    assert np.array_equal(host(us[0]), host(alone[0])) and np.array_equal(host(us[2]), host(alone[1]))


@pytest.mark.parametrize("bad", [(0.8, 0.0, 0.9), (0.8, -0.25, 0.9), (np.inf, 0.85, 0.9), (np.nan, 0.85, 0.9)])
def test_nonpositive_airlight(bad):
    require_gpu()
    import paper_2506_08793_amd as d
    I, t, A = _clean(24, 40, 75)
    Ab = np.array(bad, dtype=np.float32)
    say(f"airlight {bad}")
    # front end with a given A: every output is NaN
    pr = d.dehaze_prior(ctx(), dev(I), A_in=dev(Ab), outputs=("t_d", "t", "lam", "phi"))
    for k in ("t_d", "t", "lam", "phi"):
        assert np.isnan(host(pr[k])).all(), k
    # the solve reports it
    with pytest.raises(d.DehazeError) as e:
        d.dehaze_solve(ctx(), dev(I), dev(t), dev(Ab))
    assert e.value.code == ENONFINITE
    # and the batch flags that image only
    p = d.dehaze_params_default(max_outer=3000)
    _, st, _, _ = d.dehaze_batch(ctx(), [dev(I), dev(I)], params=p, t=[dev(t), dev(t)], A=[dev(A), dev(Ab)],
                                 allow_nonfinite=True)
    assert [s["status"] for s in st] == [0, ENONFINITE]
