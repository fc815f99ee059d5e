"""Pins of the FP64 latency-network reference: its gradient against central
finite differences, special cases with closed forms, and Adam's first step."""
import numpy as np

from oracle import mlp


def _net(F=7, H=9, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.n_params(F, H)) * 0.5
    return p, F, H, rng


def test_param_layout_roundtrip():
    p, F, H, _ = _net()
    assert np.array_equal(mlp.pack(*mlp.unpack(p, F, H)), p)
    assert mlp.n_params(F, H) == H * F + 2 * H + H * H + H + 1


def test_gradient_matches_central_differences():
    p, F, H, rng = _net()
    x = rng.standard_normal((5, F))
    t = rng.standard_normal(5)
    g, L = mlp.grad(p, F, H, x, t)
    assert abs(L - mlp.loss(p, F, H, x, t)) < 1e-12
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss(p + e, F, H, x, t) - mlp.loss(p - e, F, H, x, t)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-6 * max(1.0, np.max(np.abs(g)))


def test_all_active_network_is_affine():
    # positive weights, biases and inputs keep every ReLU active, so the
    # network is the affine map w3^T W2 W1 x + w3^T (W2 b1 + b2) + b3
    rng = np.random.default_rng(3)
    F, H = 4, 6
    W1, b1 = rng.uniform(0.1, 1, (H, F)), rng.uniform(0.1, 1, H)
    W2, b2 = rng.uniform(0.1, 1, (H, H)), rng.uniform(0.1, 1, H)
    w3, b3 = rng.standard_normal(H), 0.25
    p = mlp.pack(W1, b1, W2, b2, w3, b3)
    x = rng.uniform(0, 1, (3, F))
    want = x @ (w3 @ W2 @ W1) + w3 @ (W2 @ b1 + b2) + b3
    assert np.allclose(mlp.forward(p, F, H, x), want, rtol=1e-13, atol=1e-13)
    # and the gradient of the output bias is the mean residual times two
    t = np.zeros(3)
    g, _ = mlp.grad(p, F, H, x, t)
    assert abs(g[-1] - 2 * np.mean(want)) < 1e-12


def test_dead_network_outputs_bias():
    F, H = 3, 5
    p = np.zeros(mlp.n_params(F, H))
    p[-1] = 1.5
    assert np.all(mlp.forward(p, F, H, np.ones((4, F))) == 1.5)


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(1)
    p = rng.standard_normal(20)
    g = rng.standard_normal(20)
    q, m, v = mlp.adam_step(p, np.zeros(20), np.zeros(20), g, 1, lr=0.01, eps=0.0)
    assert np.allclose(q - p, -0.01 * np.sign(g), rtol=0, atol=1e-15)
