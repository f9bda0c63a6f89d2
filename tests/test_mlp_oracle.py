"""Pins of the warm-start network oracle: bf16 rounding against its bit-level
definition, and the analytic gradient against central differences of the
loss (in float64, without quantisation, so the finite differences are
meaningful)."""
from __future__ import annotations

import numpy as np

from oracle import mlp
from oracle import mlp as om


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


def _f32_sum_shuffled(terms, rng):
    """fp32 sum of the last axis's terms in a random order, one rounding per
    addition (a device's accumulation in some order)."""
    order = rng.permutation(terms.shape[-1])
    acc = np.zeros(terms.shape[:-1], np.float32)
    for k in order:
        acc = (acc + terms[..., k].astype(np.float32)).astype(np.float32)
    return acc


def test_layer_interval_holds_for_any_summation_order():
    """A simulated device that sums the fp32 products of each layer in a
    random order lands inside layer_interval() for every element, while its
    bf16 roundings do differ from the oracle's somewhere (the bound is
    needed)."""
    rng = np.random.default_rng(0)
    theta = om.init_params(3)
    parts = om.unpack(theta)
    X = rng.standard_normal((64, 32)).astype(np.float32)
    h = om.bf16(X).astype(np.float64)
    differ = 0
    for li, (W, b) in enumerate(parts):
        Wq = om.bf16(W).astype(np.float32)
        prods = (h.astype(np.float32)[:, :, None] * Wq[None, :, :]).transpose(0, 2, 1)  # exact in fp32
        z = (_f32_sum_shuffled(prods, rng) + b.astype(np.float32)).astype(np.float64)
        hidden = li < len(parts) - 1
        v, lo, hi = om.layer_interval(h, W, b, hidden)
        dev = om.bf16(np.maximum(z, 0).astype(np.float32)).astype(np.float64) if hidden else z
        assert np.all((dev >= lo) & (dev <= hi)), li
        differ += int(np.count_nonzero(dev != v))
        h = dev if hidden else h
    assert differ > 0


def test_grad_bound_holds_for_any_summation_order():
    """The backward pass of a simulated device (the exact dZ, products summed
    over the rows in a random fp32 order, bf16 roundings of the masked
    products) lies inside grad_bound() seeded with its activations."""
    rng = np.random.default_rng(1)
    theta = om.init_params(4)
    parts = om.unpack(theta)
    N = 40
    X = rng.standard_normal((N, 32)).astype(np.float32)
    T = rng.standard_normal((N, 4)).astype(np.float32)
    acts = [om.bf16(X).astype(np.float64)]
    h = acts[0]
    for li, (W, b) in enumerate(parts):
        z = (h @ om.bf16(W).astype(np.float64)).astype(np.float32) + b
        if li < len(parts) - 1:
            h = om.bf16(np.maximum(z, 0)).astype(np.float64)
            acts.append(h)
        else:
            Y = z.astype(np.float32)
    want, bound = om.grad_bound(theta, X, T, acts=acts, Y=Y)
    dz = om.bf16(np.float32(2.0 / (N * 4)) * (Y - T)).astype(np.float32)
    grads = []
    for li in range(len(parts) - 1, -1, -1):
        W, _ = parts[li]
        hl = acts[li].astype(np.float32)
        gW = _f32_sum_shuffled(hl.T[:, None, :] * dz.T[None, :, :], rng)  # (in, out) over rows
        gb = _f32_sum_shuffled(dz.T, rng)
        grads.append((gW, gb))
        if li > 0:
            Wq = om.bf16(W).astype(np.float32)
            dh = _f32_sum_shuffled(dz[:, None, :] * Wq[None, :, :], rng)  # (rows, in) over out
            dz = om.bf16(np.where(acts[li] > 0, dh, 0.0).astype(np.float32)).astype(np.float32)
    grads.reverse()
    got = np.concatenate([np.concatenate([a.ravel(), b]) for a, b in grads]).astype(np.float64)
    assert np.all(np.abs(got - want) <= bound)
