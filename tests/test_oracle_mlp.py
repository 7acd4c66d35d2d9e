"""Pins of the FP64 MLP oracle: its gradient equals central finite
differences of its loss (with unrounded weights, where the loss is smooth),
and BF16 rounding is round-to-nearest-even."""
import numpy as np

from oracle import mlp


def test_bf16_round_ties_and_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159265], dtype=np.float32)
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # exact tie below -> even mantissa (1.0)
    assert r[2] == 1.0 + 2 ** -7            # 1.5 ulp rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    width = [5, 7, 6, 3]
    n = mlp.param_count(width)
    p = rng.normal(0, 0.5, n)
    X = rng.normal(size=(9, 5))
    Y = rng.normal(size=(9, 3))
    loss, g = mlp.loss_grad(p, width, X, Y, round_weights=False)
    h = 1e-6
    num = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        lp, _ = mlp.loss_grad(p + e, width, X, Y, round_weights=False)
        lm, _ = mlp.loss_grad(p - e, width, X, Y, round_weights=False)
        num[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-9)


def test_planted_wrong_activation_derivative_is_caught():
    """A gradient with the SiLU derivative replaced by sigmoid fails the check."""
    rng = np.random.default_rng(1)
    width = [3, 4, 2]
    p = rng.normal(0, 0.7, mlp.param_count(width))
    X = rng.normal(size=(5, 3))
    Y = rng.normal(size=(5, 2))
    pred, cache = mlp.forward(p, width, X, round_weights=False)
    d = 2 * (pred - Y) / pred.size
    a_in, z, W = cache[1]
    g_hidden = d @ W.T
    s = 1 / (1 + np.exp(-cache[0][1]))
    wrong = (cache[0][0].T @ (g_hidden * s)).reshape(-1)
    _, g = mlp.loss_grad(p, width, X, Y, round_weights=False)
    right = g[: 3 * 4]
    assert np.abs(wrong - right).max() > 1e-3
