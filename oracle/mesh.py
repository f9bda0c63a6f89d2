"""Evaluation oracle (numpy): finest-grid resampling of leaf values, the
marching-cubes vertex set, and the quantisation error of Eq. 7.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
evaluation leg, never by the product path. Shares nothing with the HIP
library.

The vertex set of marching cubes is unique given the field: every edge
between two neighbouring finest-voxel centres whose values straddle the
iso-value (one below, one not) carries one vertex at the linear zero
crossing. How a cell joins its vertices into triangles is a choice, so the
triangles are checked for validity elsewhere, not compared.
Arithmetic (fp32, one IEEE operation at a time): t = (iso - v0) / (v1 - v0);
the coordinate along the edge is ((index + 0.5) + t) * h, the others
(index + 0.5) * h, h = 2^-D.
"""
from __future__ import annotations

import numpy as np

from . import morton_decode


def dense_from_leaves(keys, levels, u, D: int) -> np.ndarray:
    """u on the finest grid [z, y, x]: every voxel takes the value of the leaf containing it."""
    G = 1 << D
    out = np.empty((G, G, G), np.float32)
    x, y, z = morton_decode(keys)
    s = 1 << (D - np.asarray(levels, dtype=np.int64))
    for i in range(len(u)):
        out[z[i]:z[i] + s[i], y[i]:y[i] + s[i], x[i]:x[i] + s[i]] = u[i]
    return out


def _morton_encode(x, y, z) -> np.ndarray:
    x, y, z = (np.asarray(a, dtype=np.uint64) for a in (x, y, z))
    k = np.zeros(np.broadcast(x, y, z).shape, np.uint64)
    for b in range(10):
        k |= ((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
        k |= ((y >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + 1)
        k |= ((z >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + 2)
    return k


def dense_box(keys, levels, u, D: int, origin, shape) -> np.ndarray:
    """The finest-grid field on the box of `shape` (nz, ny, nx) voxels at
    `origin` (x, y, z): every voxel takes u of the leaf containing it, the
    last leaf in Morton order whose key is at most the voxel's code."""
    ox, oy, oz = origin
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(oz, oz + nz), np.arange(oy, oy + ny), np.arange(ox, ox + nx),
                             indexing="ij")
    code = _morton_encode(xx, yy, zz)
    i = np.searchsorted(np.asarray(keys, dtype=np.uint64), code, side="right") - 1
    return np.asarray(u, dtype=np.float32)[i]


def crossing_vertices(dense: np.ndarray, iso: float, D: int, origin=(0, 0, 0)):
    """Edge ids (3 * ((z G + y) G + x) + axis of the lower voxel), sorted, and
    their vertex positions (N, 3) float32 in world coordinates, of the edges
    whose two voxels lie in `dense`: the whole finest grid (G^3), or a box of
    it whose first voxel is `origin` (x, y, z)."""
    G = 1 << D
    h = np.float32(2.0 ** -D)
    iso = np.float32(iso)
    below = dense < iso
    nz, ny, nx = dense.shape
    ox, oy, oz = origin
    zz, yy, xx = np.meshgrid(np.arange(oz, oz + nz), np.arange(oy, oy + ny), np.arange(ox, ox + nx),
                             indexing="ij")
    ids, pos = [], []
    for axis in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        ax = 2 - axis  # array axis of the grid axis (arrays are [z, y, x])
        sl_lo[ax] = slice(0, dense.shape[ax] - 1)
        sl_hi[ax] = slice(1, dense.shape[ax])
        lo, hi = tuple(sl_lo), tuple(sl_hi)
        m = below[lo] != below[hi]
        v0 = dense[lo][m]
        v1 = dense[hi][m]
        t = (iso - v0) / (v1 - v0)
        X, Y, Z = xx[lo][m], yy[lo][m], zz[lo][m]
        c = [(X.astype(np.float32) + np.float32(0.5)), (Y.astype(np.float32) + np.float32(0.5)),
             (Z.astype(np.float32) + np.float32(0.5))]
        c[axis] = c[axis] + t
        p = np.stack([ci * h for ci in c], axis=1).astype(np.float32)
        e = 3 * ((Z.astype(np.uint64) * G + Y.astype(np.uint64)) * G + X.astype(np.uint64)) + np.uint64(axis)
        ids.append(e)
        pos.append(p)
    ids = np.concatenate(ids)
    pos = np.concatenate(pos)
    order = np.argsort(ids)
    return ids[order], pos[order]


def quantisation_error(keys, levels, u, dense: np.ndarray, D: int) -> float:
    """Eq. 7: sum over leaves of |u(n) - mean of dense over the voxels of n| (double)."""
    x, y, z = morton_decode(keys)
    s = 1 << (D - np.asarray(levels, dtype=np.int64))
    d = dense.astype(np.float64)
    tot = 0.0
    for i in range(len(u)):
        blk = d[z[i]:z[i] + s[i], y[i]:y[i] + s[i], x[i]:x[i] + s[i]]
        tot += abs(float(u[i]) - blk.sum() / blk.size)
    return tot
