"""Pins of the FP64 surrogate reference: a library convolution, finite differences,
adjoint identities and a library optimiser."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U


def test_conv3x3_matches_torch_circular_conv():
    """conv3x3 equals torch's conv2d on a circularly padded input (cross-correlation)."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 9, 7, 5))
    w = rng.standard_normal((6, 3, 3, 5))
    b = rng.standard_normal(6)
    ours = U.conv3x3(x, w, b)
    xt = torch.tensor(x).permute(0, 3, 1, 2)
    wt = torch.tensor(w).permute(0, 3, 1, 2)
    ref = F.conv2d(F.pad(xt, (1, 1, 1, 1), mode="circular"), wt, torch.tensor(b))
    assert np.allclose(ours, ref.permute(0, 2, 3, 1).numpy(), atol=1e-12)


def test_conv3x3_backward_is_adjoint():
    """<conv(x), g> - <bias term> is bilinear: the input and weight gradients satisfy
    <dx, x> = <dw, w> = <conv(x) - b, g> for the linear part."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 8, 4))
    w = rng.standard_normal((3, 3, 3, 4))
    g = rng.standard_normal((2, 6, 8, 3))
    lin = (U.conv3x3(x, w, np.zeros(3)) * g).sum()
    dx, dw, db = U.conv3x3_backward(x, w, g)
    assert np.isclose((dx * x).sum(), lin, rtol=1e-12)
    assert np.isclose((dw * w).sum(), lin, rtol=1e-12)
    assert np.allclose(db, g.sum(axis=(0, 1, 2)))


def test_pool_upsample_adjoints_and_silu():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((1, 4, 6, 3))
    b = rng.standard_normal((1, 8, 12, 3))
    assert np.isclose((U.upsample2(a) * b).sum(), (a * U.upsample2_backward(b)).sum())
    assert np.isclose((U.avgpool2(b) * a).sum(), (b * U.avgpool2_backward(a)).sum())
    assert np.allclose(U.avgpool2(U.upsample2(a)), a)
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(U.silu_grad(z), (U.silu(z + h) - U.silu(z - h)) / (2 * h), atol=1e-8)


def test_network_gradient_finite_differences():
    """The hand-written backward pass of the whole U-Net agrees with central finite
    differences of the MSE loss (float64, 16x16 input so that three poolings fit)."""
    rng = np.random.default_rng(3)
    params = U.init_weights(5)
    x = rng.standard_normal((1, 16, 16, U.IN_CH))
    y = rng.standard_normal((1, 16, 16, U.OUT_CH))
    out, cache = U.forward(params, x)
    loss, dout = U.mse(out, y)
    grads = U.backward(params, cache, dout)
    h = 1e-5
    picks = [("e0a", 0), ("e0b", 0), ("b3b", 0), ("u2", 0), ("d2a", 0), ("u0", 0),
             ("d0b", 0), ("head", 0), ("e1a", 1), ("d1a", 1), ("head", 1)]
    for name, which in picks:
        arr = params[name][which]
        g = grads[name][which]
        for _ in range(3):
            idx = tuple(rng.integers(0, n) for n in arr.shape)
            old = arr[idx]
            arr[idx] = old + h
            lp = U.mse(U.forward(params, x)[0], y)[0]
            arr[idx] = old - h
            lm = U.mse(U.forward(params, x)[0], y)[0]
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, which, idx, fd, g[idx])


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    p0 = rng.standard_normal(10)
    pt = torch.nn.Parameter(torch.tensor(p0.copy()))
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(10), np.zeros(10)
    for t in range(1, 6):
        g = rng.standard_normal(10)
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = U.adam(p, g, m, v, t, 1e-2)
    assert np.allclose(p, pt.detach().numpy(), atol=1e-12)
