"""Pins of the warm-start network oracle against torch's float64 CPU
convolution, autograd and Adam (library routines) and finite differences."""
import numpy as np
import torch
import torch.nn.functional as F

from oracle import cnn_ref as c


def _weights(seed, layers=c.LAYERS, scale=0.2):
    rng = np.random.default_rng(seed)
    return [(rng.normal(0, scale, size=(co, ci, 3, 3)), rng.normal(0, 0.1, size=co)) for ci, co in layers]


def test_conv3x3_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 9, 7))
    Wt = rng.normal(size=(4, 5, 3, 3))
    b = rng.normal(size=4)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(Wt), torch.from_numpy(b), padding=1).numpy()
    assert np.max(np.abs(c.conv3x3(x, Wt, b) - ref)) < 1e-12


def test_forward_backward_match_autograd():
    layers = ((7, 6), (6, 6), (6, 3))
    ws = _weights(1, layers)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 7, 8, 10))
    target = rng.normal(size=(2, 3, 8, 10))
    y, cache = c.forward(x, ws)
    loss, gy = c.mse(y, target)
    grads = c.backward(cache, ws, gy)
    tw = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in ws]
    h = torch.from_numpy(x)
    for k, (W, b) in enumerate(tw):
        h = F.conv2d(h, W, b, padding=1)
        if k != len(tw) - 1:
            h = torch.relu(h)
    tl = torch.mean((h - torch.from_numpy(target)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-12
    assert np.max(np.abs(y - h.detach().numpy())) < 1e-12
    for (dW, db), (W, b) in zip(grads, tw):
        assert np.max(np.abs(dW - W.grad.numpy())) < 1e-12
        assert np.max(np.abs(db - b.grad.numpy())) < 1e-12


def test_backward_finite_differences():
    layers = ((7, 4), (4, 3))
    ws = _weights(3, layers)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(1, 7, 5, 6))
    target = rng.normal(size=(1, 3, 5, 6))

    def loss_of(wlist):
        y, _ = c.forward(x, wlist)
        return c.mse(y, target)[0]

    y, cache = c.forward(x, ws)
    grads = c.backward(cache, ws, c.mse(y, target)[1])
    h = 1e-6
    for k in range(len(ws)):
        for idx in [(0, 0, 1, 1), (1, 2, 0, 2), (2, 3, 2, 0)]:
            if idx[0] >= ws[k][0].shape[0] or idx[1] >= ws[k][0].shape[1]:
                continue
            wp = [(W.copy(), b.copy()) for W, b in ws]
            wm = [(W.copy(), b.copy()) for W, b in ws]
            wp[k][0][idx] += h
            wm[k][0][idx] -= h
            fd = (loss_of(wp) - loss_of(wm)) / (2 * h)
            assert abs(fd - grads[k][0][idx]) < 1e-7 * max(1.0, abs(fd))


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=(3, 4))
    gs = [rng.normal(size=(3, 4)) for _ in range(5)]
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for s, g in enumerate(gs, start=1):
        p, m, v = c.adam_step(p, g, m, v, s, lr=1e-2)
        opt.zero_grad()
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.max(np.abs(p - tp.detach().numpy())) < 1e-12


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-5, 5, size=10000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(c.round_bf16(x), ref)


def test_features_layout():
    I = np.arange(3 * 2 * 4, dtype=np.float32).reshape(3, 2, 4)
    t = np.full((2, 4), 0.25)
    f = c.features(I, t, [0.8, 0.85, 0.9])
    assert f.shape == (7, 2, 4)
    assert np.array_equal(f[:3], I) and np.all(f[3] == 0.25) and np.all(f[6] == 0.9)
