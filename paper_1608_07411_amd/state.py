"""State blobs (otf_export_state / otf_import_state) on the host: parsing,
and cutting one aligned cube out of a state as a state of its own.

The blob layout (little-endian): "OTF1", u32 version 1, the 40-byte parameter
block, i64 iteration, i32 view count, i32 0; per view an i64 node count and
the view octree's nodes {u32 key, u8 level, u8 leaf, u16 0, f32 S, u32 cnt}
in (level, key) order; an i64 leaf count and the fused octree's leaves
{u32 key, u8 level, u8[3] 0, f32 u, ubar, p_x, p_y, p_z} in key order. Keys
are Morton codes of the min-corner finest voxel (x in bit 0).

No arithmetic of the method happens here: a cut keeps every value the method
reads (a view node's mean F = S / cnt and weight W = cnt / volume) exactly.
"""
from __future__ import annotations

import struct

import numpy as np

NODE = np.dtype([("key", "<u4"), ("level", "u1"), ("leaf", "u1"), ("pad", "<u2"), ("S", "<f4"), ("cnt", "<u4")])
LEAF = np.dtype([("key", "<u4"), ("level", "u1"), ("pad", "u1", (3,)), ("v", "<f4", (5,))])
HEADER = 8 + 40 + 8 + 8


def parse(blob: bytes):
    """(max_depth, view node arrays, leaf array) of a state blob (views)."""
    D = struct.unpack_from("<i", blob, 8)[0]
    at = HEADER - 8
    nv = struct.unpack_from("<i", blob, at)[0]
    at += 8
    views = []
    for _ in range(nv):
        n = struct.unpack_from("<q", blob, at)[0]
        at += 8
        views.append(np.frombuffer(blob, NODE, n, at))
        at += n * NODE.itemsize
    nl = struct.unpack_from("<q", blob, at)[0]
    at += 8
    return D, views, np.frombuffer(blob, LEAF, nl, at)


def _view_cover(nodes: np.ndarray, D: int, cube_level: int, n_cubes: int):
    """Per cube at cube_level of one view octree: the level of the deepest
    node containing the cube (cube_level if the octree stores a node for it),
    or -1 if that node is a coarser leaf whose count is not a multiple of the
    volume ratio (its weight over the cube would not be an integer count)."""
    k = nodes["key"].astype(np.int64)
    lv = nodes["level"].astype(np.int64)
    sh = 3 * (D - cube_level)
    out = np.full(n_cubes, -1, np.int8)
    # coarser leaves first, deeper ones overwrite: the deepest containing node wins
    for L in range(cube_level):
        sel = (lv == L) & (nodes["leaf"] == 1)
        span = 1 << (3 * (cube_level - L))
        for kk, c in zip((k[sel] >> sh).tolist(), nodes["cnt"][sel].tolist()):
            out[kk:kk + span] = L if c % span == 0 else -1
    at = lv == cube_level
    out[(k[at] >> sh)] = cube_level
    return out


def crop(blob: bytes, cube_level: int, M=None, min_leaves: int = 10000, max_leaves: int | None = None):
    """State blob of one aligned cube at cube_level, re-rooted as a domain of
    depth D - cube_level. Every view must store a node for the cube, or its
    deepest node containing the cube must be a leaf whose count divides
    exactly by the volume ratio 8^k: that leaf becomes the view's root with
    count cnt / 8^k and sum S / 8^k (exact in fp32), so that its mean and
    weight are unchanged.
    Among such cubes tiled by at least min_leaves leaves (at most max_leaves),
    the one whose mean observation count per leaf (M, per leaf of the whole
    state) is closest to the whole octree's, else the one with the most
    leaves. Returns (blob, leaf count, cube index). Raises ValueError if no
    cube qualifies."""
    D, views, leaves = parse(blob)
    sh = 3 * (D - cube_level)
    n_cubes = 1 << (3 * cube_level)
    cube_of = leaves["key"].astype(np.int64) >> sh
    counts = np.bincount(cube_of, minlength=n_cubes)
    coarse = np.bincount(cube_of[leaves["level"] < cube_level], minlength=n_cubes) > 0
    ok = (counts >= min_leaves) & ~coarse
    if max_leaves is not None:
        ok &= counts <= max_leaves
    covers = [_view_cover(nodes, D, cube_level, n_cubes) for nodes in views]
    for cv in covers:
        ok &= cv >= 0
    if not ok.any():
        raise ValueError(f"no level-{cube_level} cube can be cut exactly")
    if M is not None:
        msum = np.bincount(cube_of, weights=np.asarray(M, np.float64), minlength=n_cubes)
        mean = np.where(ok, msum / np.maximum(counts, 1), np.inf)
        best = int(np.argmin(np.abs(mean - float(np.mean(M)))))
    else:
        best = int(np.argmax(np.where(ok, counts, -1)))
    mask = (1 << sh) - 1
    out = bytearray(blob[:HEADER])
    struct.pack_into("<i", out, 8, D - cube_level)
    for nodes, cv in zip(views, covers):
        k = nodes["key"].astype(np.int64)
        lv = nodes["level"].astype(np.int64)
        L = int(cv[best])
        if L == cube_level:
            sub = nodes[(lv >= cube_level) & ((k >> sh) == best)].copy()
            sub["level"] -= cube_level
            sub["key"] = (sub["key"].astype(np.int64) & mask).astype(np.uint32)
        else:  # a coarser leaf: its count and sum over the cube's share of it
            src = nodes[(lv == L) & ((k >> (3 * (D - L))) == (best << sh) >> (3 * (D - L)))]
            assert len(src) == 1 and src["leaf"][0] == 1
            kk = 3 * (cube_level - L)
            sub = np.zeros(1, NODE)
            sub["leaf"] = 1
            sub["cnt"] = int(src["cnt"][0]) >> kk
            sub["S"] = np.float32(src["S"][0]) * np.float32(2.0 ** -kk)
        out += struct.pack("<q", len(sub)) + sub.tobytes()
    sel = leaves[cube_of == best].copy()
    sel["level"] -= cube_level
    sel["key"] = (sel["key"].astype(np.int64) & mask).astype(np.uint32)
    out += struct.pack("<q", len(sel)) + sel.tobytes()
    return bytes(out), len(sel), best
