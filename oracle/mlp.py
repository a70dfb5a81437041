"""Plain FP64 multilayer perceptron: the reference for the surrogate's GPU kernels.  Test
infrastructure only.

Network: h_0 = x; for hidden layers l = 0 .. L-2: z_l = h_l W_l^T + b_l, h_{l+1} = tanh(z_l);
output y = h_{L-1} W_{L-1}^T + b_{L-1} (linear).  W_l has shape (out_l, in_l).
Loss: mean squared error over the batch and the outputs, L = sum (y - t)^2 / (batch * n_out).
Gradients by the chain rule, written out layer by layer (no automatic differentiation).
Parameters are packed as W_0 (row-major), b_0, W_1, b_1, ... in that order.
"""
from __future__ import annotations

import numpy as np


def shapes(widths):
    return [(widths[i + 1], widths[i]) for i in range(len(widths) - 1)]


def n_params(widths) -> int:
    return sum(o * i + o for o, i in shapes(widths))


def unpack(params, widths):
    out, pos = [], 0
    for o, i in shapes(widths):
        W = params[pos:pos + o * i].reshape(o, i)
        pos += o * i
        b = params[pos:pos + o]
        pos += o
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def init(widths, seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights and zero biases."""
    rng = np.random.default_rng(seed)
    layers = []
    for o, i in shapes(widths):
        lim = 1.0 / np.sqrt(i)
        layers.append((rng.uniform(-lim, lim, size=(o, i)), np.zeros(o)))
    return pack(layers)


def forward(params, widths, x):
    """Returns the output and the list of layer inputs h_l (for the backward pass)."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    h = np.asarray(x, dtype=np.float64)
    hs = [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.tanh(z) if li < len(layers) - 1 else z
        hs.append(h)
    return h, hs


def loss_and_grad(params, widths, x, t):
    """MSE loss and its gradient with respect to the packed parameters."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    y, hs = forward(params, widths, x)
    t = np.asarray(t, dtype=np.float64)
    B, nout = y.shape
    loss = float(np.sum((y - t) ** 2) / (B * nout))
    dz = 2.0 * (y - t) / (B * nout)          # d loss / d z_{L-1} (linear output)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        h_in = hs[li]
        grads[li] = (dz.T @ h_in, dz.sum(axis=0))
        if li > 0:
            dh = dz @ W                        # d loss / d h_li
            dz = dh * (1.0 - hs[li] ** 2)      # tanh' = 1 - tanh^2, hs[li] = tanh(z_{li-1})
    return loss, pack(grads)


def input_grad(params, widths, x, w_out):
    """Gradient with respect to x of sum_k w_out[k] y[:, k] (per sample)."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    y, hs = forward(params, widths, x)
    dz = np.tile(np.asarray(w_out, dtype=np.float64), (y.shape[0], 1))
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        dh = dz @ W
        dz = dh * (1.0 - hs[li] ** 2) if li > 0 else dh
    return y, dz


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
