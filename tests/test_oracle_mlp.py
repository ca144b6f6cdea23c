"""Pins of the oracle's FP64 MLP (the learned early-stop network, 15 -> 64 ->
64 -> 1, ReLU, MSE) against central finite differences and torch FP64
autograd, of its Adam step against the first-step closed form, and of the
early-stop features on a hand-worked search state."""
import math

import numpy as np
import torch

import oracle

IN, H = 15, 64


def _params(seed):
    rng = np.random.default_rng(seed)
    n = oracle.mlp_nparams(IN, H)
    assert n == 15 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5249
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


def test_stop_features_worked_example():
    """A pool of 12 entries with distances 3, 4, ..., 14 (ranks past the
    pool take its last entry, 14), start node at distance 63, 50 neighbour
    entries read over 10 expansions."""
    f = oracle.stop_features(np.arange(3, 15, dtype=np.float32), 63.0, 50, 10)
    assert f.shape == (15,)
    assert f[0] == math.log(4.0)                      # ln(1 + 3)
    assert f[1] == 3.0 / 12.0                         # d_0 / d_9 (rank 9 holds 12)
    assert f[2] == math.log(64.0)
    assert abs(f[3] - math.log(4.0 / 64.0)) < 1e-15
    want = [5, 6, 8, 13, 15, 15, 15, 15, 15, 15]      # 1 + d at ranks 1, 2, 4, 9, then 14 (clamped)
    for j, w in enumerate(want):
        assert abs(f[4 + j] - math.log(w / 4.0)) < 1e-15, j
    assert f[14] == 5.0
    # degenerate: a one-entry pool at distance 0 and no expansions
    g = oracle.stop_features(np.zeros(1, np.float32), 0.0, 0, 0)
    assert g[1] == 1.0 and g[14] == 0.0 and (g[[0, 2, 3]] == 0).all() and (g[4:14] == 0).all()


def test_fp16_forward_equals_fp64_forward_on_representable_values():
    """With the query form's shape (131 -> 64 -> 64 -> 1), integer inputs and
    weights in {-1, 0, 1} (8 nonzero first-layer weights per unit) and small
    integer biases, every input, weight and hidden activation is an integer
    below 2048 in magnitude, exact in FP16: the FP16-inference forward then
    equals the FP64 forward of the oracle's C code."""
    n_in, h = 131, 64
    rng = np.random.default_rng(3)
    W1 = np.zeros((h, n_in))
    for j in range(h):
        W1[j, rng.choice(n_in, 8, replace=False)] = rng.choice([-1.0, 1.0], 8)
    b1 = rng.integers(-2, 3, size=h).astype(float)
    W2 = rng.integers(-1, 2, size=(h, h)).astype(float)
    b2 = rng.integers(-2, 3, size=h).astype(float)
    W3 = rng.integers(-1, 2, size=h).astype(float)
    P = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [0.5]])
    assert P.size == oracle.mlp_nparams(n_in, h)
    X = rng.integers(-1, 2, size=(8, n_in)).astype(float)
    _, _, want = oracle.mlp_loss_grad(P, X, None, n_in, h)
    got = oracle.mlp_forward_fp16(P, X, n_in, h)
    assert np.abs(want).max() > 4 and len(set(want.tolist())) > 4
    assert (got == want).all(), (got, want)


def test_fp16_forward_rounding_points():
    """1 -> 1 -> 1 -> 1 networks: the input, the weights and each hidden
    activation are rounded to FP16 to nearest, ties to even (spacing 2^-10
    just above 1), overflow gives inf, ReLU clips negatives; biases are not
    rounded."""
    def net(w1=1.0, b1=0.0, w2=1.0, b2=0.0, w3=1.0, b3=0.0):
        return np.array([w1, b1, w2, b2, w3, b3])

    f = lambda P, x: float(oracle.mlp_forward_fp16(P, np.array([[x]]), 1, 1)[0])
    u = 2.0 ** -10
    assert f(net(), 1 + u / 2) == 1.0                    # tie -> even (1)
    assert f(net(), 1 + 3 * u / 2) == 1 + 2 * u          # tie -> even (1 + 2u)
    assert f(net(), 1 + 0.6 * u) == 1 + u                # nearest
    assert f(net(), 7e4) == math.inf                     # beyond FP16's largest finite value
    assert f(net(), -3.0) == 0.0
    assert f(net(w1=1 + u / 2), 1.0) == 1.0              # weight rounded
    assert f(net(b1=u / 2), 1.0) == 1.0                  # first activation rounded (1 + u/2 -> 1)
    assert f(net(b2=u / 2), 1.0) == 1.0                  # second activation rounded
    assert f(net(b3=u / 4), 1.0) == 1 + u / 4            # output bias not rounded
    assert f(net(w3=-1 - u / 2), 1.0) == -1.0            # output weight rounded


def test_query_form_inputs():
    q = np.array([1.5, -2.0, 0.25], np.float32)
    x = oracle.stop_query_inputs(q, np.arange(3, 15, dtype=np.float32), 16)
    assert x.shape == (6,)
    assert (x[:3] == q).all() and x[3] == math.log(4.0) and x[4] == 3.0 / 12.0 and x[5] == 16.0
    y = oracle.stop_query_inputs(q, np.array([0.0], np.float32), 0)
    assert (y[3:] == [0.0, 1.0, 0.0]).all()
