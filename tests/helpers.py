"""Shared test utilities: blob field edits, leaf geometry, dense resampling."""
from __future__ import annotations

import math
import struct

import numpy as np

from oracle import morton_decode

TAU32 = float(np.float32(1.0 / math.sqrt(12.0)))

# byte offsets inside the state blob header
_OFF_PARAMS = 8
_PARAM_FIELDS = {  # name: (offset inside the parameter block, struct format)
    "max_depth": (0, "<i"), "delta": (4, "<f"), "eta": (8, "<f"), "spread_tau": (12, "<f"),
    "gamma": (16, "<f"), "split_tau": (20, "<f"), "join_tau": (24, "<f"),
    "restructure_every": (28, "<i"), "max_leaves": (32, "<q"),
}


def blob_set(blob: bytes, **fields) -> bytes:
    b = bytearray(blob)
    for k, v in fields.items():
        off, fmt = _PARAM_FIELDS[k]
        struct.pack_into(fmt, b, _OFF_PARAMS + off, v)
    return bytes(b)


def blob_get(blob: bytes, name: str):
    off, fmt = _PARAM_FIELDS[name]
    return struct.unpack_from(fmt, blob, _OFF_PARAMS + off)[0]


def parse_views(blob: bytes):
    """Per-view node lists from a state blob: list of structured arrays."""
    at = 8 + 40 + 8
    n_views = struct.unpack_from("<i", blob, at)[0]
    at += 8
    dt = np.dtype([("key", "<u4"), ("level", "u1"), ("leaf", "u1"), ("pad", "<u2"), ("S", "<f4"), ("cnt", "<u4")])
    views = []
    for _ in range(n_views):
        n = struct.unpack_from("<q", blob, at)[0]
        at += 8
        views.append(np.frombuffer(blob, dtype=dt, count=n, offset=at).copy())
        at += n * dt.itemsize
    nl = struct.unpack_from("<q", blob, at)[0]
    at += 8
    ldt = np.dtype([("key", "<u4"), ("level", "u1"), ("pad", "u1", (3,)), ("u", "<f4"), ("ubar", "<f4"),
                    ("p", "<f4", (3,))])
    leaves = np.frombuffer(blob, dtype=ldt, count=nl, offset=at).copy()
    return views, leaves


def blob_set_leaves(blob: bytes, u=None, ubar=None, p=None) -> bytes:
    """Copy of a state blob with the leaves' u, ubar or p replaced (leaf order)."""
    at = 8 + 40 + 8
    n_views = struct.unpack_from("<i", blob, at)[0]
    at += 8
    for _ in range(n_views):
        n = struct.unpack_from("<q", blob, at)[0]
        at += 8 + 16 * n
    nl = struct.unpack_from("<q", blob, at)[0]
    at += 8
    ldt = np.dtype([("key", "<u4"), ("level", "u1"), ("pad", "u1", (3,)), ("u", "<f4"), ("ubar", "<f4"),
                    ("p", "<f4", (3,))])
    b = bytearray(blob)
    leaves = np.frombuffer(b, dtype=ldt, count=nl, offset=at)
    for name, v in (("u", u), ("ubar", ubar), ("p", p)):
        if v is not None:
            leaves[name] = np.asarray(v, dtype=np.float32).reshape(leaves[name].shape)
    return bytes(b)


def leaf_boxes(keys, levels, max_depth):
    x, y, z = morton_decode(keys)
    s = (1 << (max_depth - levels.astype(np.int64)))
    return x, y, z, s


def to_dense(keys, levels, values, max_depth):
    """Piecewise-constant resampling of per-leaf values to the finest grid [z, y, x]."""
    G = 1 << max_depth
    out = np.zeros((G, G, G))
    x, y, z, s = leaf_boxes(keys, levels, max_depth)
    for i in range(len(keys)):
        out[z[i]:z[i] + s[i], y[i]:y[i] + s[i], x[i]:x[i] + s[i]] = values[i]
    return out


def plane_volumes(n_views, max_depth, seed, p_unobs=0.0, noise=0.05):
    """Per-view TSDF-like volumes from random planes (unbalanced trees)."""
    rng = np.random.default_rng(seed)
    G = 1 << max_depth
    zz, yy, xx = np.meshgrid(*(np.arange(G) + 0.5,) * 3, indexing="ij")
    f = np.empty((n_views, G, G, G), np.float32)
    w = np.empty((n_views, G, G, G), np.uint8)
    for v in range(n_views):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        c = rng.uniform(0.3, 0.7, 3) * G
        d = (xx - c[0]) * n[0] + (yy - c[1]) * n[1] + (zz - c[2]) * n[2]
        val = np.clip(d / rng.uniform(1.0, 3.0), -1, 1) + noise * rng.normal(size=d.shape)
        f[v] = np.clip(val, -1, 1)
        w[v] = rng.uniform(size=d.shape) >= p_unobs
    return f, w


def base_params(max_depth, **over):
    p = dict(max_depth=max_depth, delta=0.1, eta=1.0, spread_tau=0.1, gamma=1e-2, split_tau=0.5,
             join_tau=0.9, restructure_every=1, max_leaves=0)
    p.update(over)
    return p


def blob_volumes(n_views, max_depth, seed, p_unobs=0.0, noise=0.02):
    """Per-view volumes of a small sphere-like blob (thin band, unbalanced tree)."""
    rng = np.random.default_rng(seed)
    G = 1 << max_depth
    zz, yy, xx = np.meshgrid(*(np.arange(G) + 0.5,) * 3, indexing="ij")
    c = rng.uniform(0.35, 0.65, 3) * G
    r = rng.uniform(0.15, 0.3) * G
    f = np.empty((n_views, G, G, G), np.float32)
    w = np.empty((n_views, G, G, G), np.uint8)
    for v in range(n_views):
        cc = c + rng.normal(scale=0.3, size=3)
        d = np.sqrt((xx - cc[0]) ** 2 + (yy - cc[1]) ** 2 + (zz - cc[2]) ** 2) - r
        val = np.clip(d / 1.5, -1, 1) + noise * rng.normal(size=d.shape) * (np.abs(d) < 2)
        f[v] = np.clip(val, -1, 1)
        w[v] = rng.uniform(size=d.shape) >= p_unobs
    return f, w
