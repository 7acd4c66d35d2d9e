"""FP64 reference of the surrogate MLP (test oracle).

Same function as the library's kernels: layer l maps width[l] -> width[l+1]
as y = x W_l + b_l, SiLU (x * sigmoid(x)) on hidden layers, linear output,
loss = mean over all entries of (prediction - target)^2.  Weights are used
with the values they have after rounding to BF16 (round to nearest even), as
the kernels read them; everything else is FP64.  The parameter vector is laid
out layer by layer as W_l (row-major) then b_l.

Test infrastructure only (see the package docstring).  Parity: pinned against
central finite differences of its own loss (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np


def param_count(width):
    return sum((width[l] + 1) * width[l + 1] for l in range(len(width) - 1))


def bf16_round(x):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(params, width):
    out, off = [], 0
    for l in range(len(width) - 1):
        I, O = width[l], width[l + 1]
        W = params[off: off + I * O].reshape(I, O)
        b = params[off + I * O: off + (I + 1) * O]
        out.append((W, b))
        off += (I + 1) * O
    return out


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, width, X, round_weights=True):
    """Prediction and the per-layer (input, pre-activation) cache."""
    layers = unpack(np.asarray(params, dtype=np.float64), width)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        Wq = bf16_round(W) if round_weights else W
        z = a @ Wq + b
        cache.append((a, z, Wq))
        a = z * _sig(z) if l + 1 < len(layers) else z
    return a, cache


def loss_grad(params, width, X, Y, round_weights=True):
    """MSE loss and its gradient with respect to params (weights treated as
    their rounded values, i.e. the straight-through gradient the kernels
    compute)."""
    pred, cache = forward(params, width, X, round_weights)
    n = pred.size
    d = pred - np.asarray(Y, dtype=np.float64)
    loss = float((d * d).sum() / n)
    grad_out = 2.0 * d / n
    grads = []
    g = grad_out
    L = len(cache)
    for l in range(L - 1, -1, -1):
        a_in, z, Wq = cache[l]
        if l + 1 < L:
            s = _sig(z)
            g = g * (s * (1.0 + z * (1.0 - s)))
        gW = a_in.T @ g
        gb = g.sum(axis=0)
        grads.append(np.concatenate([gW.reshape(-1), gb]))
        g = g @ Wq.T
    return loss, np.concatenate(grads[::-1])
