"""Pins of the MLP oracle (the learned warm start) against closed forms,
finite differences and torch's independent float64 implementation."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp

SMALL = (5, 8, 8, 8, 4)


def _theta(sizes, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mlp.param_count(sizes))


def test_param_count_matches_layer_sizes():
    assert mlp.param_count() == 5 * 128 + 128 + 2 * (128 * 128 + 128) + 4 * 128 + 4 == 34308
    assert mlp.param_count(SMALL) == 5 * 8 + 8 + 2 * (64 + 8) + 32 + 4


def test_silu_closed_forms():
    assert mlp.silu(0.0) == 0.0
    assert mlp.silu(math.log(3.0)) == pytest.approx(0.75 * math.log(3.0), rel=1e-15)
    x = np.linspace(-30, 30, 121)
    # x sigma(x) - (-x) sigma(-x) = x (sigma(x) + sigma(-x)) = x
    np.testing.assert_allclose(mlp.silu(x) - mlp.silu(-x), x, rtol=1e-14, atol=1e-14)
    assert mlp.silu_prime(0.0) == 0.5
    assert mlp.silu_prime(math.log(3.0)) == pytest.approx(0.75 * (1 + math.log(3.0) / 4), rel=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.silu_prime(x), (mlp.silu(x + h) - mlp.silu(x - h)) / (2 * h), rtol=1e-8,
                               atol=1e-9)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = _theta(SMALL, 1)
    x = rng.normal(size=(37, 5))
    t = rng.normal(size=(37, 4))

    def loss(th):
        y, _ = mlp.forward(th, x, SMALL)
        return mlp.mse(y, t)[0]

    y, cache = mlp.forward(theta, x, SMALL)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(theta, cache, dy, SMALL)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(len(theta)):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (loss(theta + e) - loss(theta - e)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)
    big = np.abs(fd) > 1e-3 * np.abs(fd).max()
    np.testing.assert_allclose(g[big], fd[big], rtol=1e-6)


def _torch_net(theta, sizes):
    layers = []
    for l, (W, b) in enumerate(mlp.unpack(theta, sizes)):
        lin = torch.nn.Linear(W.shape[1], W.shape[0], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W.copy()))
            lin.bias.copy_(torch.from_numpy(b.copy()))
        layers.append(lin)
        if l + 1 < len(sizes) - 1:
            layers.append(torch.nn.SiLU())
    return torch.nn.Sequential(*layers)


def test_forward_and_backward_match_torch_float64():
    rng = np.random.default_rng(2)
    theta = _theta(mlp.SIZES, 3, scale=0.15)
    x = rng.normal(size=(64, 5))
    t = rng.normal(size=(64, 4))
    net = _torch_net(theta, mlp.SIZES)
    xt = torch.from_numpy(x)
    yt = net(xt)
    loss_t = torch.nn.functional.mse_loss(yt, torch.from_numpy(t))
    loss_t.backward()
    ref = torch.cat([torch.cat([m.weight.grad.reshape(-1), m.bias.grad]) for m in net
                     if isinstance(m, torch.nn.Linear)]).numpy()
    y, cache = mlp.forward(theta, x)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-13)
    loss, dy = mlp.mse(y, t)
    assert loss == pytest.approx(loss_t.item(), rel=1e-13)
    g = mlp.backward(theta, cache, dy)
    assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mse_of_exact_prediction_is_zero():
    y = np.arange(12.0).reshape(3, 4)
    loss, dy = mlp.mse(y, y)
    assert loss == 0.0 and not dy.any()


def test_adam_first_step_and_constant_gradient_closed_form():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    lr, eps = 1e-2, 1e-8
    m = v = np.zeros(4)
    # with a constant gradient the bias-corrected moments are g and g^2 at
    # every step, so each step moves by lr g / (|g| + eps)
    for t in range(1, 6):
        p_new, m, v = mlp.adam_step(p, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(p - p_new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
        p = p_new


def test_adam_matches_torch_over_varying_gradients():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=50)
    grads = rng.normal(size=(7, 50))
    pt = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, t, 3e-3)
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_features_geometry():
    r = 0.3
    dirs = np.random.default_rng(6).normal(size=(20, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    on_surface = 0.5 + r * dirs
    f = mlp.features(on_surface, r, 0.7)
    np.testing.assert_allclose(f[:, 3], 0.0, atol=1e-15)
    np.testing.assert_allclose(f[:, :3], r * dirs, atol=1e-15)
    assert (f[:, 4] == 0.7).all()
    c = mlp.features(np.array([[0.5, 0.5, 0.5]]), r, 0.7)
    np.testing.assert_allclose(c[0, :4], [0, 0, 0, -r])
    # the cell is periodic: shifting by lattice vectors changes nothing, and
    # the farthest point from the centre is a cell corner at sqrt(3)/2
    pts = np.random.default_rng(7).uniform(0, 1, (50, 3))
    shifted = pts + np.random.default_rng(8).integers(-2, 3, (50, 3))
    np.testing.assert_allclose(mlp.features(shifted, r, 0.7), mlp.features(pts, r, 0.7), atol=1e-12)
    assert np.all(np.abs(mlp.features(pts, r, 0.7)[:, :3]) <= 0.5)
    corner = mlp.features(np.zeros((1, 3)), r, 0.7)
    assert corner[0, 3] == pytest.approx(math.sqrt(3) / 2 - r, rel=1e-15)


def test_to_state_boundary_and_gauge():
    y = np.arange(40.0).reshape(10, 4)
    v, p = mlp.to_state(y, 6, 2.0, 3.0)
    assert not v[:, 6:].any()
    np.testing.assert_allclose(v[:, :6], 2.0 * y[:6, :3].T)
    assert abs(p.mean()) < 1e-12
    np.testing.assert_allclose(np.diff(p), 3.0 * np.diff(y[:, 3]))
