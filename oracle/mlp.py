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


# ---------------------------------------------------------------------------
# Per-element error bounds: how far a device that rounds the same values to
# bf16 as above, but accumulates its fp32 sums in another order (any order,
# any split into partial sums), can lie from this oracle. Interval arithmetic
# through every layer: the standard bound |fl(sum) - sum| <= g_n sum |terms|,
# g_n = n u / (1 - n u), u = 2^-24, for each fp32 sum of n terms, one unit
# roundoff per other fp32 operation, and bf16 rounding handled exactly as a
# monotone map (the device's value lies between the bf16 roundings of its
# interval's ends, so where the whole interval rounds to one bf16 value the
# two sides agree exactly).
# ---------------------------------------------------------------------------
_U = 2.0 ** -24


def _g(n: int) -> float:
    return n * _U / (1.0 - n * _U)


def _f32_down(x):
    x = np.asarray(x, np.float64)
    y = x.astype(np.float32)
    return np.where(y.astype(np.float64) > x, np.nextafter(y, np.float32(-np.inf)), y)


def _f32_up(x):
    x = np.asarray(x, np.float64)
    y = x.astype(np.float32)
    return np.where(y.astype(np.float64) < x, np.nextafter(y, np.float32(np.inf)), y)


def _bf16_spread(v, lo, hi):
    """Largest distance from v (the oracle's bf16 value) to the bf16 roundings
    of an interval [lo, hi] that contains the device's unrounded value."""
    a = bf16(_f32_down(lo)).astype(np.float64)
    b = bf16(_f32_up(hi)).astype(np.float64)
    v = np.asarray(v, np.float64)
    return np.maximum(b - v, v - a)


def _sum_bound(E_in, absA, absB, E_B, n_terms):
    """Bound on |sum' - sum| of products A B when A carries errors E_in, B
    errors E_B (both elementwise), with an fp32 sum of n_terms terms in any
    order on the device."""
    spread = E_in @ absB + absA @ E_B + E_in @ E_B
    mags = (absA + E_in) @ (absB + E_B)
    return spread + _g(n_terms) * mags


def forward_bound(theta: np.ndarray, X: np.ndarray):
    """Outputs of forward() and a bound on |Y_device - Y| per element; also
    the hidden activations and their bounds (for grad_bound)."""
    layers = unpack(np.asarray(theta, dtype=np.float32))
    h = bf16(X).astype(np.float64)
    E = np.zeros_like(h)
    acts, errs = [h], [E]
    Y = None
    for li, (W, b) in enumerate(layers):
        Wq = bf16(W).astype(np.float64)
        s = h @ Wq
        z = s.astype(np.float32) + b.astype(np.float32)  # the oracle's value
        Ez = _sum_bound(E, np.abs(h), np.abs(Wq), np.zeros_like(Wq), W.shape[0] + 64)
        Ez = Ez + 3 * _U * (np.abs(s) + np.abs(b) + Ez)  # roundings of the sum and the bias add
        z64 = z.astype(np.float64)
        if li < len(layers) - 1:
            hn = bf16(np.maximum(z, 0.0)).astype(np.float64)
            E = _bf16_spread(hn, np.maximum(z64 - Ez, 0.0), np.maximum(z64 + Ez, 0.0))
            h = hn
            acts.append(h)
            errs.append(E)
        else:
            Y, E = z64, Ez
    return Y, E, acts, errs


def layer_interval(h: np.ndarray, W: np.ndarray, b: np.ndarray, hidden: bool):
    """One layer from exact bf16 inputs h: the oracle's output and the interval
    [lo, hi] that holds the output of any device accumulating the same fp32
    products in another order (hidden layers: bf16(ReLU(z)) values; the output
    layer: fp32 z)."""
    h = np.asarray(h, np.float64)
    Wq = bf16(W).astype(np.float64)
    s = h @ Wq
    z = (s.astype(np.float32) + np.asarray(b, np.float32)).astype(np.float64)
    Ez = _g(Wq.shape[0] + 64) * (np.abs(h) @ np.abs(Wq)) + 3 * _U * (np.abs(s) + np.abs(b))
    if not hidden:
        return z, z - Ez, z + Ez
    v = bf16(np.maximum(z, 0.0).astype(np.float32)).astype(np.float64)
    lo = bf16(_f32_down(np.maximum(z - Ez, 0.0))).astype(np.float64)
    hi = bf16(_f32_up(np.maximum(z + Ez, 0.0))).astype(np.float64)
    return v, lo, hi


def grad_bound(theta: np.ndarray, X: np.ndarray, T: np.ndarray, acts=None, Y=None):
    """The gradient of loss_and_grad() and a bound on |grad_device - grad| per
    element, for a device that forms dZ = bf16(fp32(2/n) * fp32(Y - T)) and the
    products and column sums as above in any accumulation order. Given the
    device's own activations (acts: bf16(X) and the 3 hidden layers) and
    outputs Y, the bound starts from them exactly (only the backward pass's
    sums and bf16 roundings differ); otherwise from forward_bound()."""
    layers = unpack(np.asarray(theta, dtype=np.float32))
    if acts is None:
        Yo, EY, acts, errs = forward_bound(theta, X)
        _, g = loss_and_grad(theta, X, T)
    else:
        acts = [np.asarray(a, np.float64) for a in acts]
        errs = [np.zeros_like(a) for a in acts]
        Yo, EY = np.asarray(Y, np.float64), np.zeros(np.shape(Y))
        g = None
    N = X.shape[0]
    n = N * Yo.shape[1]
    c = 2.0 / n
    if g is None:
        # the device's dZ exactly: fp32 difference, fp32 product, bf16
        dz = bf16(np.float32(c) * (np.asarray(Y, np.float32) - np.asarray(T, np.float32))).astype(np.float64)
        Edz = np.zeros_like(dz)
    else:
        d = Yo - np.asarray(T, np.float64)
        lo = (d - EY) * c
        hi = (d + EY) * c
        slack = 4 * _U * (np.abs(d) + EY) * c
        dz = bf16((c * d).astype(np.float32)).astype(np.float64)
        Edz = _bf16_spread(dz, lo - slack, hi + slack)
    grads, bounds = [], []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        Wq = bf16(W).astype(np.float64)
        h, Eh = acts[li], errs[li]
        gW = h.T @ dz
        EgW = _sum_bound(Eh.T, np.abs(h).T, np.abs(dz), Edz, N + 1024) + 2 * _U * np.abs(gW)
        gb = dz.sum(axis=0)
        Egb = Edz.sum(axis=0) + _g(N + 1024) * (np.abs(dz) + Edz).sum(axis=0) + 2 * _U * np.abs(gb)
        grads.append((gW, gb))
        bounds.append((EgW, Egb))
        if li > 0:
            dh = dz @ Wq.T
            Edh = _sum_bound(Edz, np.abs(dz), np.abs(Wq).T, np.zeros_like(Wq.T), Wq.shape[1] + 64)
            Edh = Edh + 2 * _U * (np.abs(dh) + Edh)
            on = h > 0
            sure = np.where(on, h - Eh > 0, h + Eh <= 0)  # the device's mask agrees for sure
            dzn = bf16(np.where(on, dh, 0.0).astype(np.float32)).astype(np.float64)
            lo = np.where(sure, np.where(on, dh - Edh, 0.0), np.minimum(0.0, dh - Edh))
            hi = np.where(sure, np.where(on, dh + Edh, 0.0), np.maximum(0.0, dh + Edh))
            Edz = _bf16_spread(dzn, lo, hi)
            dz = dzn
    grads.reverse()
    bounds.reverse()
    if g is None:
        g = np.concatenate([np.concatenate([a.ravel(), b]) for a, b in grads])
    Eg = np.concatenate([np.concatenate([a.ravel(), b]) for a, b in bounds])
    return g, Eg
