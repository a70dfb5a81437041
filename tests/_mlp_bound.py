"""Element-by-element error bars for the surrogate network's BF16 matrix-core arithmetic, and a
numpy emulation of that arithmetic (test infrastructure only).

The GPU rounds both operands of every product to BF16 (8 significant bits, round to nearest
even: relative error in [-u_b, u_b], u_b = 2^-8, variance at most u_b^2/3 per operand) and
accumulates in FP32.  A worst-case bound (sum of absolute values) grows by the norm of |W| at
every layer and is vacuous for a 256-wide, four-product network, so the bars follow the
probabilistic model of rounding error (independent, zero-mean errors per operation; Higham and
Mary, "A new approach to probabilistic rounding error analysis", SIAM J. Sci. Comput. 2019):
for C = A B with inputs carrying independent errors of variances vA, vB,

    var(C_ij) = sum_k [vA_ik B_kj^2 + A_ik^2 vB_kj + (2 u_b^2 / 3 + K u_f^2) (A_ik B_kj)^2],

tanh is linearised (var_h = (1 - h^2)^2 var_z), and the derivative 1 - h^2 moves with h.  The
variances are propagated through the layers of oracle/mlp.py's network with the FP64 oracle's
own activations, and the bar of each element is LAMBDA standard deviations plus a floor of a
few FP32 units of the element's scale.
"""
from __future__ import annotations

import numpy as np

U_B = 2.0 ** -8
U_F = 2.0 ** -24
LAMBDA = 6.0
R2 = 2.0 * U_B * U_B / 3.0


def gemm_var(A, vA, B, vB, K):
    A2, B2 = A * A, B * B
    return vA @ B2 + A2 @ vB + (R2 + K * U_F * U_F) * (A2 @ B2)


def _layers(params, widths):
    from oracle import mlp
    return mlp.unpack(np.asarray(params, dtype=np.float64), widths)


def _bar(v, scale):
    return LAMBDA * np.sqrt(v) + 16 * U_F * scale


def forward_var(params, widths, x):
    """(y, var_y, hs, vs): oracle output and layer inputs with the variances of their errors."""
    layers = _layers(params, widths)
    h = np.asarray(x, dtype=np.float64)
    v = np.zeros_like(h)
    hs, vs = [h], [v]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        vz = gemm_var(h, v, W.T, np.zeros_like(W.T), W.shape[1])
        if li < len(layers) - 1:
            h = np.tanh(z)
            v = vz * (1.0 - h * h) ** 2
        else:
            h, v = z, vz
        hs.append(h)
        vs.append(v)
    return h, v, hs, vs


def forward_bar(params, widths, x):
    y, v, _, _ = forward_var(params, widths, x)
    return y, _bar(v, np.abs(y).max())


def _back(layers, dz, vdz, hs, vs, stop_at_input):
    """Backward pass with variances: yields (li, dz, vdz, h_in, v_in) for every layer, top down."""
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        yield li, dz, vdz
        dh = dz @ W
        vdh = gemm_var(dz, vdz, W, np.zeros_like(W), W.shape[0])
        if li > 0:
            h_in, v_in = hs[li], vs[li]
            g = 1.0 - h_in * h_in
            dz = dh * g
            vdz = vdh * g * g + dh * dh * 4.0 * h_in * h_in * v_in
        elif stop_at_input:
            yield -1, dh, vdh


def grad_bar(params, widths, x, t):
    """Bars of the packed parameter gradient (oracle/mlp.py's layout)."""
    layers = _layers(params, widths)
    y, vy, hs, vs = forward_var(params, widths, x)
    B, nout = y.shape
    dz = 2.0 * (y - np.asarray(t, dtype=np.float64)) / (B * nout)
    vdz = 4.0 * vy / (B * nout) ** 2
    out = [None] * len(layers)
    for li, dzl, vdzl in _back(layers, dz, vdz, hs, vs, False):
        gW = dzl.T @ hs[li]
        vW = gemm_var(dzl.T, vdzl.T, hs[li], vs[li], B)
        gb = dzl.sum(axis=0)
        vb = vdzl.sum(axis=0) + B * U_F * U_F * (dzl * dzl).sum(axis=0)
        out[li] = (_bar(vW, np.abs(gW).max()), _bar(vb, np.abs(gb).max()))
    return np.concatenate([np.concatenate([eW.reshape(-1), eb]) for eW, eb in out])


def input_grad_bar(params, widths, x, w_out):
    """(bar_y, bar_dx): bars of the output and of the input gradient of sum_k w_out[k] y[:, k]."""
    layers = _layers(params, widths)
    y, vy, hs, vs = forward_var(params, widths, x)
    dz = np.tile(np.asarray(w_out, dtype=np.float64), (y.shape[0], 1))
    dx = vdx = None
    for li, d, v in _back(layers, dz, np.zeros_like(dz), hs, vs, True):
        if li == -1:
            dx, vdx = d, v
    return _bar(vy, np.abs(y).max()), _bar(vdx, np.abs(dx).max())


# ------------------------------------------------------------------ emulation of the GPU arithmetic
def bf16(a):
    """Round float32 values to BF16 (round to nearest, ties to even), returned as float32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def emulate_forward(params, widths, x, fault=None):
    """The network as the GPU computes it: FP32 weights and activations, BF16 operands, FP32
    accumulation (numpy float32 products), FP32 bias and tanh.  fault(li, z) may alter a layer's
    product (a planted kernel mistake)."""
    layers = _layers(params, widths)
    h = np.asarray(x, dtype=np.float32)
    for li, (W, b) in enumerate(layers):
        z = bf16(h) @ bf16(np.asarray(W, dtype=np.float32)).T
        if fault is not None:
            fault(li, z)
        z = z + np.asarray(b, dtype=np.float32)
        h = np.tanh(z) if li < len(layers) - 1 else z
    return h.astype(np.float64)


def emulate_loss_grad(params, widths, x, t):
    """Packed parameter gradient of the MSE loss as the GPU computes it (same arithmetic as
    emulate_forward; the backward products also take BF16 operands)."""
    layers = _layers(params, widths)
    h = np.asarray(x, dtype=np.float32)
    hs = [h]
    for li, (W, b) in enumerate(layers):
        z = bf16(h) @ bf16(np.asarray(W, dtype=np.float32)).T + np.asarray(b, dtype=np.float32)
        h = np.tanh(z) if li < len(layers) - 1 else z
        hs.append(h)
    y = hs[-1]
    B, nout = y.shape
    dz = (np.float32(2.0 / (B * nout)) * (y - np.asarray(t, dtype=np.float32))).astype(np.float32)
    out = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W = np.asarray(layers[li][0], dtype=np.float32)
        out[li] = (bf16(dz).T @ bf16(hs[li]), dz.sum(axis=0, dtype=np.float32))
        if li > 0:
            dz = (bf16(dz) @ bf16(W)) * (np.float32(1.0) - hs[li] * hs[li])
    return np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in out]).astype(np.float64)
