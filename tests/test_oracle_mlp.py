"""Pins of the binary64 selector-network oracle: finite differences, torch autograd (a library
special case), Adam's closed form under a constant gradient, and convergence on a toy fit."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp


def _data(n, seed):
    g = synth.rng(seed)
    X = g.standard_normal((n, 4))
    Y = np.stack([np.sin(X[:, 0]) + X[:, 1], X[:, 2] * 0.5, -X[:, 3], X[:, 0] * X[:, 1]], axis=1)
    return X, Y


def test_param_count_and_pack_roundtrip():
    p = synth.mlp_init(0).astype(np.float64)
    assert p.size == synth.mlp_param_count() == 4 * 64 + 64 + 64 * 64 + 64 + 64 * 4 + 4 == 4740
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_gradient_central_differences():
    X, Y = _data(24, 1)
    p = synth.mlp_init(3).astype(np.float64)
    loss, g = mlp.loss_and_grad(p, X, Y)
    rs = synth.rng(2)
    idx = rs.choice(p.size, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, Y)[0] - mlp.loss_and_grad(p - e, X, Y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    X, Y = _data(50, 4)
    p = synth.mlp_init(5).astype(np.float64)
    loss, g = mlp.loss_and_grad(p, X, Y)
    layers = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
              for W, b in mlp.unpack(p)]
    h = torch.tensor(X)
    for li, (W, b) in enumerate(layers):
        z = torch.nn.functional.linear(h, W, b)
        h = torch.relu(z) if li < 2 else z
    tl = torch.mean((h - torch.tensor(Y)) ** 2)
    tl.backward()
    tg = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy()]) for W, b in layers])
    assert abs(tl.item() - loss) <= 1e-14 * abs(loss)
    assert np.max(np.abs(tg - g)) <= 1e-13 * max(1.0, np.max(np.abs(g)))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, bias-corrected m_hat = g and v_hat = g^2 at every step,
    so each update is -lr * g / (|g| + eps)."""
    p = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -7.0])
    m = np.zeros(5)
    v = np.zeros(5)
    for t in range(1, 11):
        p2, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-2)
        assert np.allclose(p2 - p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        p = p2


def test_adam_matches_torch():
    p0 = synth.mlp_init(7).astype(np.float64)
    X, Y = _data(64, 8)
    p, losses = mlp.train(p0, X, Y, steps=25, lr=1e-3)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(25):
        opt.zero_grad()
        loss, g = mlp.loss_and_grad(tp.detach().numpy(), X, Y)
        tp.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(tp.detach().numpy() - p)) <= 1e-12


def test_training_reduces_loss():
    X, Y = _data(200, 9)
    mu, sd = mlp.standardize_stats(X)
    p, losses = mlp.train(synth.mlp_init(1).astype(np.float64), (X - mu) / sd, Y, steps=300, lr=3e-3)
    assert losses[-1] < 0.25 * losses[0]


def test_standardize_zero_std():
    X = np.array([[1.0, 2.0], [1.0, 4.0]])
    mu, sd = mlp.standardize_stats(X)
    assert list(mu) == [1.0, 3.0] and list(sd) == [1.0, 1.0]
