"""Pins of the FP64 MLP oracle (oracle/mlp.py): central finite differences for the parameter
and input gradients (the backward pass against the forward pass), the closed form of a
single linear layer (least-squares gradient), zero-weight networks, and the first Adam step."""
import numpy as np

from oracle import mlp


def test_parameter_gradient_matches_finite_differences():
    widths = [7, 12, 9, 2]
    rng = np.random.default_rng(0)
    p = mlp.init(widths, seed=1) + 0.05 * rng.standard_normal(mlp.n_params(widths))
    x = rng.uniform(-1, 1, size=(5, 7))
    t = rng.standard_normal((5, 2))
    _, g = mlp.loss_and_grad(p, widths, x, t)
    h = 1e-6
    idx = rng.choice(p.size, size=60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, widths, x, t)[0] - mlp.loss_and_grad(p - e, widths, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_input_gradient_matches_finite_differences():
    widths = [5, 16, 16, 2]
    rng = np.random.default_rng(2)
    p = mlp.init(widths, seed=3)
    x = rng.uniform(-1, 1, size=(3, 5))
    w = np.array([1.0, -0.5])
    _, gx = mlp.input_grad(p, widths, x, w)
    h = 1e-6
    for s in range(3):
        for k in range(5):
            xp, xm = x.copy(), x.copy()
            xp[s, k] += h
            xm[s, k] -= h
            fp = mlp.forward(p, widths, xp)[0][s] @ w
            fm = mlp.forward(p, widths, xm)[0][s] @ w
            assert abs((fp - fm) / (2 * h) - gx[s, k]) <= 1e-8


def test_single_linear_layer_is_least_squares():
    widths = [4, 3]
    rng = np.random.default_rng(4)
    W = rng.standard_normal((3, 4))
    b = rng.standard_normal(3)
    p = mlp.pack([(W, b)])
    X = rng.standard_normal((6, 4))
    T = rng.standard_normal((6, 3))
    loss, g = mlp.loss_and_grad(p, widths, X, T)
    R = X @ W.T + b - T
    assert abs(loss - np.sum(R * R) / 18) < 1e-14
    gW = 2.0 / 18 * R.T @ X
    gb = 2.0 / 18 * R.sum(axis=0)
    np.testing.assert_allclose(g, mlp.pack([(gW, gb)]), rtol=0, atol=1e-14)


def test_zero_weights_output_is_bias():
    widths = [3, 8, 2]
    p = np.zeros(mlp.n_params(widths))
    p[-2:] = [0.7, -0.2]
    y, _ = mlp.forward(p, widths, np.ones((4, 3)))
    np.testing.assert_allclose(y, np.tile([0.7, -0.2], (4, 1)), atol=0)


def test_first_adam_step_moves_by_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    p1, _, _ = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), step=1, lr=0.01)
    np.testing.assert_allclose(p1, -0.01 * np.sign(g), rtol=1e-4)
