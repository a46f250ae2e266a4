"""Pins of the learned-fill oracle (oracle/unet.py) against library routines
(torch CPU float64 ops and autograd), finite differences and closed forms."""
from __future__ import annotations

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U



@pytest.fixture(autouse=True)
def _float64_default():
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def rand_params(rng, scale=1.0):
    return [rng.normal(0, scale * np.sqrt(2.0 / (9 * cin)), size=(9, cout, cin)) for _, cin, cout in U.LAYERS]


def to_torch_w(w):
    """[9, Cout, Cin] -> torch [Cout, Cin, 3, 3]."""
    return torch.from_numpy(w.reshape(3, 3, w.shape[1], w.shape[2]).transpose(2, 3, 0, 1).copy())


def nchw(x):
    return torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)))


def nhwc(t):
    return t.detach().numpy().transpose(0, 2, 3, 1)


def torch_net(params, x):
    """The same architecture written with torch.nn.functional (float64)."""
    W = [to_torch_w(w) for w in params]
    c = lambda v, i: F.conv2d(v, W[i], padding=1)  # noqa: E731
    r = F.relu
    e0 = r(c(r(c(x, 0)), 1))
    e1 = r(c(r(c(F.avg_pool2d(e0, 2), 2)), 3))
    e2 = r(c(r(c(F.avg_pool2d(e1, 2), 4)), 5))
    e3 = r(c(r(c(F.avg_pool2d(e2, 2), 6)), 7))
    up = lambda v: F.interpolate(v, scale_factor=2, mode="nearest")  # noqa: E731
    d2 = r(c(r(c(torch.cat([r(c(up(e3), 8)), e2], 1), 9)), 10))
    d1 = r(c(r(c(torch.cat([r(c(up(d2), 11)), e1], 1), 12)), 13))
    d0 = r(c(r(c(torch.cat([r(c(up(d1), 14)), e0], 1), 15)), 16))
    return c(d0, 17)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 5000),
                        np.array([1.0, -1.0, 0.0, 1.00390625, 1.01171875, 3.0e38, -2.5e-3])]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16(x), want)


def test_conv_and_its_gradients_match_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 5))
    w = rng.normal(size=(9, 4, 5))
    g = rng.normal(size=(2, 7, 9, 4))
    xt = nchw(x).requires_grad_(True)
    wt = to_torch_w(w).requires_grad_(True)
    yt = F.conv2d(xt, wt, padding=1)
    assert np.allclose(U.conv3x3(x, w), nhwc(yt), rtol=1e-12, atol=1e-12)
    yt.backward(nchw(g))
    assert np.allclose(U.conv3x3_grad_input(g, w), nhwc(xt.grad), rtol=1e-12, atol=1e-12)
    gw = wt.grad.numpy().transpose(2, 3, 0, 1).reshape(9, 4, 5)
    assert np.allclose(U.conv3x3_grad_weight(x, g), gw, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_match_torch():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 6, 3))
    assert np.allclose(U.avgpool2(x), nhwc(F.avg_pool2d(nchw(x), 2)))
    assert np.allclose(U.upsample2(x), nhwc(F.interpolate(nchw(x), scale_factor=2, mode="nearest")))
    g = rng.normal(size=(2, 4, 3, 3))
    xt = nchw(x).requires_grad_(True)
    F.avg_pool2d(xt, 2).backward(nchw(g))
    assert np.allclose(U.avgpool2_grad(g), nhwc(xt.grad))
    g2 = rng.normal(size=(2, 16, 12, 3))
    xt = nchw(x).requires_grad_(True)
    F.interpolate(xt, scale_factor=2, mode="nearest").backward(nchw(g2))
    assert np.allclose(U.upsample2_grad(g2), nhwc(xt.grad))


def test_network_forward_and_backward_match_torch_autograd():
    rng = np.random.default_rng(3)
    params = rand_params(rng)
    x = rng.uniform(0, 1, size=(2, 16, 16, 5))
    res, cache = U.forward(params, x, rounding=False)
    xt = nchw(x)
    Wt = [torch.from_numpy(p).requires_grad_(True) for p in params]
    yt = torch_net([w for w in params], xt)
    assert np.allclose(res, nhwc(yt), rtol=1e-10, atol=1e-12)
    g = rng.normal(size=res.shape)
    gw, _ = U.backward(params, cache, g, rounding=False)
    # autograd through the torch net with the weights as leaves
    Wl = [to_torch_w(p).requires_grad_(True) for p in params]

    def net_w(W):
        c = lambda v, i: F.conv2d(v, W[i], padding=1)  # noqa: E731
        r = F.relu
        up = lambda v: F.interpolate(v, scale_factor=2, mode="nearest")  # noqa: E731
        e0 = r(c(r(c(xt, 0)), 1))
        e1 = r(c(r(c(F.avg_pool2d(e0, 2), 2)), 3))
        e2 = r(c(r(c(F.avg_pool2d(e1, 2), 4)), 5))
        e3 = r(c(r(c(F.avg_pool2d(e2, 2), 6)), 7))
        d2 = r(c(r(c(torch.cat([r(c(up(e3), 8)), e2], 1), 9)), 10))
        d1 = r(c(r(c(torch.cat([r(c(up(d2), 11)), e1], 1), 12)), 13))
        d0 = r(c(r(c(torch.cat([r(c(up(d1), 14)), e0], 1), 15)), 16))
        return c(d0, 17)

    net_w(Wl).backward(nchw(g))
    for i, (a, b) in enumerate(zip(gw, Wl)):
        want = b.grad.numpy().transpose(2, 3, 0, 1).reshape(a.shape)
        assert np.allclose(a, want, rtol=1e-9, atol=1e-12), U.LAYERS[i][0]
    del Wt


def test_gradient_matches_finite_differences():
    """Central differences of the full masked-L1 loss (no rounding, float64),
    on a reduced input, for a few weights of several layers."""
    rng = np.random.default_rng(4)
    params = rand_params(rng)
    N, H, W = 1, 16, 16
    rgba = rng.integers(0, 256, size=(N, H, W, 4), dtype=np.uint8)
    depth = np.exp(rng.uniform(np.log(0.3), np.log(50), size=(N, H, W))).astype(np.float32)
    mask = (rng.random((N, H, W)) < 0.4).astype(np.uint8)
    target = rng.integers(0, 256, size=(N, H, W, 4), dtype=np.uint8)
    x = U.make_input(rgba, depth, mask)
    res, cache = U.forward(params, x, rounding=False)
    loss, g = U.masked_l1(res, rgba, mask, target)
    gw, _ = U.backward(params, cache, g, rounding=False)
    h = 1e-6
    for li in (0, 5, 8, 12, 16, 17):
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in params[li].shape)
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[li][idx] += h
            pm[li][idx] -= h
            num = (U.loss_of(pp, rgba, depth, mask, target, False) - U.loss_of(pm, rgba, depth, mask, target, False)) / (2 * h)
            assert abs(num - gw[li][idx]) <= 1e-5 * max(1.0, abs(num)), (U.LAYERS[li][0], idx, num, gw[li][idx])


def test_masked_l1_closed_form():
    rgba = np.zeros((1, 1, 2, 4), dtype=np.uint8)
    rgba[0, 0, 0, :3] = [100, 100, 100]
    mask = np.array([[[1, 0]]], dtype=np.uint8)
    target = np.zeros_like(rgba)
    target[0, 0, 0, :3] = [110, 90, 100]
    res = np.zeros((1, 1, 2, 3))
    loss, g = U.masked_l1(res, rgba, mask, target)
    assert abs(loss - (10 / 255 + 10 / 255 + 0) / 3) < 1e-15
    assert np.allclose(g[0, 0, 0], [-1 / 3, 1 / 3, 0]) and np.all(g[0, 0, 1] == 0)
    l0, g0 = U.masked_l1(res, rgba, np.zeros_like(mask), target)
    assert l0 == 0.0 and not g0.any()


def test_make_input_and_composite_closed_forms():
    rgba = np.array([[[[255, 0, 51, 7], [10, 20, 30, 40]]]], dtype=np.uint8)
    depth = np.array([[[0.3, np.inf]]], dtype=np.float32)
    mask = np.array([[[0, 2]]], dtype=np.uint8)
    x = U.make_input(rgba, depth, mask)
    assert np.allclose(x[0, 0, 0], [1.0, 0.0, 0.2, 0.0, 0.0], atol=1e-7)
    assert np.allclose(x[0, 0, 1], [10 / 255, 20 / 255, 30 / 255, 1.0, 1.0])
    res = np.zeros((1, 1, 2, 3))
    res[0, 0, 1] = [0.0, -1.0, 2.0]
    out = U.composite(res, rgba, mask)
    assert out[0, 0, 0].tolist() == [255, 0, 51, 7]          # not a hole: unchanged
    assert out[0, 0, 1].tolist() == [10, 0, 255, 40]         # zero residual keeps, clamps, alpha kept


def test_composite_quantisation_in_fp32():
    """Zero residual gives back every level, k/255 shifts by k (clamped), and
    an exact FP32 tie x.5 rounds to the even neighbour."""
    f = np.float32
    lv = np.arange(256, dtype=np.uint8)
    rgba = np.stack([lv, lv, lv, lv], -1)[None, None]
    mask = np.ones(rgba.shape[:3], np.uint8)
    for k in range(-5, 6):
        out = U.composite(np.full(rgba.shape[:3] + (3,), f(k) / f(255)), rgba, mask)
        assert np.array_equal(out[..., 0], np.clip(lv.astype(int) + k, 0, 255)[None, None])
        assert np.array_equal(out[..., 3], rgba[..., 3])
    for c in (10, 11, 100, 101):
        r0 = f(0.5 / 255)
        cand = r0 + np.arange(-200, 200, dtype=np.float32) * np.spacing(r0)
        tie = cand[f(255) * (f(c) / f(255) + cand) == f(c + 0.5)]
        assert tie.size > 0
        px = np.array([[[[c, c, c, 255]]]], np.uint8)
        out = U.composite(np.full((1, 1, 1, 3), tie[0]), px, np.ones((1, 1, 1), np.uint8))
        assert out[0, 0, 0, 0] == (c if c % 2 == 0 else c + 1)


def test_adamw_matches_torch():
    rng = np.random.default_rng(5)
    w0 = rng.normal(size=50)
    wt = torch.from_numpy(w0.copy()).requires_grad_(True)
    opt = torch.optim.AdamW([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        wt.grad = torch.from_numpy(g.copy())
        opt.step()
        w, m, v = U.adamw_step(w, m, v, g, step)
    assert np.allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adamw_first_step_closed_form():
    w, m, v = U.adamw_step(np.array([2.0, -1.0]), np.zeros(2), np.zeros(2), np.array([0.5, -3.0]), 1)
    # m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps) after the decay.
    assert np.allclose(w, [2.0 * (1 - 1e-5) - 1e-3 * 0.5 / (0.5 + 1e-8), -1.0 * (1 - 1e-5) + 1e-3 * 3.0 / (3.0 + 1e-8)])
