"""Pins of the oracle's FP64 MLP (the learned early-stop network, 131 -> 64 ->
64 -> 1, ReLU, MSE) against central finite differences and torch FP64
autograd, and of its Adam step against the first-step closed form."""
import numpy as np
import torch

import oracle

IN, H = 131, 64


def _params(seed):
    rng = np.random.default_rng(seed)
    n = oracle.mlp_nparams(IN, H)
    assert n == 131 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 12673
    return rng.normal(size=n) * 0.2


def test_grad_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    X = rng.normal(size=(7, IN))
    y = rng.normal(size=7)
    loss, g, _ = oracle.mlp_loss_grad(p, X, y, IN, H)
    idx = rng.choice(p.size, 300, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.mlp_loss_grad(pp, X, y, IN, H)[0] - oracle.mlp_loss_grad(pm, X, y, IN, H)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8


def test_matches_torch_autograd_fp64():
    rng = np.random.default_rng(3)
    p = _params(4)
    X = rng.normal(size=(33, IN))
    y = rng.normal(size=33)
    loss, g, yhat = oracle.mlp_loss_grad(p, X, y, IN, H)
    t = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = t[o:o + H * IN].view(H, IN); o += H * IN
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + H * H].view(H, H); o += H * H
    b2 = t[o:o + H]; o += H
    W3 = t[o:o + H]; o += H
    b3 = t[o:o + 1]
    xt = torch.tensor(X)
    out = torch.relu(torch.relu(xt @ W1.T + b1) @ W2.T + b2) @ W3 + b3
    L = ((out - torch.tensor(y)) ** 2).mean()
    L.backward()
    np.testing.assert_allclose(yhat, out.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(loss - L.item()) <= 1e-12 * abs(loss)
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    m = np.zeros(100)
    v = np.zeros(100)
    p0 = p.copy()
    oracle.adam_step(p, g, m, v, 1, lr=1e-3)
    # after bias correction m_hat = g, v_hat = g^2: step = lr * g / (|g| + eps)
    np.testing.assert_allclose(p0 - p, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
