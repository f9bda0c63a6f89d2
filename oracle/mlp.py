"""Oracle of the warm-start network (numpy).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
path. Shares nothing with the HIP library.

A per-leaf multilayer perceptron: 32 inputs -> 128 -> 128 -> 128 -> 4 outputs
(u and the 3 components of p), ReLU on the hidden layers. Weights and
activations are bfloat16 (fp32 rounded to nearest, ties to even, on the top
16 bits), products accumulate in fp32 (here: float64, then rounded to fp32,
so that only the accumulation order differs from a device), biases fp32.
Loss: mean squared error over rows and the 4 outputs.
Parameter vector layout: for each layer l, W_l (in x out, row-major) then
b_l (out).
"""
from __future__ import annotations

import numpy as np

SIZES = (32, 128, 128, 128, 4)


def n_params(sizes=SIZES) -> int:
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def bf16(x: np.ndarray) -> np.ndarray:
    """Round fp32 values to bfloat16 (nearest, ties to even), returned as fp32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def unpack(theta: np.ndarray, sizes=SIZES):
    out, at = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = theta[at:at + a * b].reshape(a, b)
        at += a * b
        bb = theta[at:at + b]
        at += b
        out.append((W, bb))
    return out


def forward(theta: np.ndarray, X: np.ndarray, quantise: bool = True):
    """Outputs (N, 4) fp32 and the hidden activations (for backward)."""
    q = bf16 if quantise else (lambda a: np.asarray(a, dtype=np.float32))
    layers = unpack(np.asarray(theta, dtype=np.float32))
    h = q(X)
    acts = [h]
    for li, (W, b) in enumerate(layers):
        z = (h.astype(np.float64) @ q(W).astype(np.float64)).astype(np.float32) + b.astype(np.float32)
        if li < len(layers) - 1:
            h = q(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, acts


def loss_and_grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray, quantise: bool = True):
    """MSE loss and its gradient with respect to theta (fp32 master weights;
    the bf16 rounding of weights is treated as the identity in the gradient,
    as training with bf16 copies of fp32 masters does)."""
    q = bf16 if quantise else (lambda a: np.asarray(a, dtype=np.float32))
    layers = unpack(np.asarray(theta, dtype=np.float32))
    Y, acts = forward(theta, X, quantise)
    N = X.shape[0]
    diff = Y.astype(np.float64) - T
    loss = float(np.mean(diff ** 2))
    dz = q((2.0 / (N * Y.shape[1]) * diff).astype(np.float32))
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h = acts[li]
        gW = (h.astype(np.float64).T @ dz.astype(np.float64)).astype(np.float32)
        gb = dz.astype(np.float64).sum(axis=0).astype(np.float32)
        grads.append((gW, gb))
        if li > 0:
            dh = (dz.astype(np.float64) @ q(W).astype(np.float64).T).astype(np.float32)
            dz = q(np.where(acts[li] > 0, dh, 0.0).astype(np.float32))
    grads.reverse()
    return loss, np.concatenate([np.concatenate([g.ravel(), b]) for g, b in grads]).astype(np.float32)


def init_params(seed: int, sizes=SIZES) -> np.ndarray:
    """He-normal weights, zero biases, from a seeded generator."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal(a * b) * np.sqrt(2.0 / a)).astype(np.float32))
        parts.append(np.zeros(b, np.float32))
    return np.concatenate(parts)
