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


def test_bf16_elementwise_bars_hold_and_catch_a_bad_tile():
    """The per-element bars of the GPU tests (tests/_mlp_bound.py) against a numpy emulation of the
    GPU's arithmetic (BF16 operands, FP32 accumulation): every output element lies inside its bar,
    the bars are tight (median below 3% of the output scale), and a 3% error in one 64 x 64 tile of
    a hidden layer's product puts some output element outside its bar, where a 2e-2 relative
    Frobenius-norm check of the output would not see it."""
    import _mlp_bound as mb
    from oracle import mlp
    widths = [9, 256, 256, 256, 2]
    rng = np.random.default_rng(11)
    p = mlp.init(widths, seed=12)
    x = rng.uniform(-1, 1, size=(300, widths[0]))
    y, bar = mb.forward_bar(p, widths, x)
    ye = mb.emulate_forward(p, widths, x)
    assert np.all(np.abs(ye - y) <= bar)
    assert np.median(bar) < 3e-2 * np.max(np.abs(y))

    def fault(li, z):
        if li == 1:
            z[64:128, 64:128] *= 1.03

    bad = mb.emulate_forward(p, widths, x, fault=fault)
    assert np.any(np.abs(bad - y) > bar)
    assert np.linalg.norm(bad - y) < 2e-2 * np.linalg.norm(y)


def test_bf16_gradient_bars_hold():
    """Every element of the emulated GPU parameter gradient lies inside its bar."""
    import _mlp_bound as mb
    from oracle import mlp
    widths = [9, 256, 256, 256, 2]
    rng = np.random.default_rng(13)
    p = mlp.init(widths, seed=14)
    x = rng.uniform(-1, 1, size=(300, widths[0]))
    t = rng.standard_normal((300, 2))
    _, g = mlp.loss_and_grad(p, widths, x, t)
    bar = mb.grad_bar(p, widths, x, t)
    ge = mb.emulate_loss_grad(p, widths, x, t)
    assert np.all(np.abs(ge - g) <= bar), float(np.max(np.abs(ge - g) / bar))


def test_bf16_bound_of_the_bf16_rounding():
    """bf16() rounds to the nearest value with 8 significant bits, ties to even."""
    import _mlp_bound as mb
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -3.0 + 2 ** -8], dtype=np.float32)
    np.testing.assert_array_equal(mb.bf16(v), np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0, -3.0], dtype=np.float32))
    r = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    rel = np.abs(mb.bf16(r) - r) / np.abs(r)
    assert rel.max() <= mb.U_B * (1 + 1e-6)
    assert rel.max() > 0.9 * mb.U_B
