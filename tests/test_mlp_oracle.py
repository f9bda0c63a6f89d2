"""Pins of the warm-start network oracle: bf16 rounding against its bit-level
definition, and the analytic gradient against central differences of the
loss (in float64, without quantisation, so the finite differences are
meaningful)."""
from __future__ import annotations

import numpy as np

from oracle import mlp


def test_bf16_rounding_bits():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.14159265], np.float32)
    r = mlp.bf16(x)
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0 + 2 ** -7)
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even) -> 1 + 2^-6
    assert r[3] == np.float32(1.0 + 2 ** -6)
    assert r[4] == -2.5 and r[5] == 0.0
    assert np.all(r.view(np.uint32) & 0xFFFF == 0)
    assert abs(r[6] - 3.14159265) < 2 ** -7 * 4


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1).astype(np.float64)
    X = rng.standard_normal((64, 32))
    T = rng.standard_normal((64, 4))
    _, g = mlp.loss_and_grad(theta.astype(np.float32), X.astype(np.float32), T, quantise=False)

    def loss(th):
        # float64 forward for the finite differences
        layers = mlp.unpack(th)
        h = X
        for li, (W, b) in enumerate(layers):
            z = h @ W + b
            h = np.maximum(z, 0) if li < len(layers) - 1 else z
        return np.mean((h - T) ** 2)

    idx = rng.choice(theta.size, 40, replace=False)
    eps = 1e-4
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (loss(tp) - loss(tm)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-3 * max(1e-3, abs(fd)) + 1e-6, (i, fd, g[i])


def test_quantised_forward_is_close_to_exact():
    rng = np.random.default_rng(2)
    theta = mlp.init_params(3)
    X = rng.standard_normal((256, 32)).astype(np.float32)
    yq, _ = mlp.forward(theta, X, True)
    ye, _ = mlp.forward(theta, X, False)
    assert np.max(np.abs(yq - ye)) < 0.05 * np.max(np.abs(ye))
