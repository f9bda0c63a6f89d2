"""Pins of the evaluation oracle (oracle/mesh.py): brute-force resampling,
closed-form vertex positions for a linear field, and the values Eq. 7 must
take for fields built from the leaves."""
from __future__ import annotations

import numpy as np

from oracle import Oracle, morton_decode
from oracle import mesh as om
from paper_1608_07411_amd import synth


def _small():
    w = synth.sphere_workload(max_depth=4, n_views=3, W=40, H=30, f=37.5)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    o.fuse(3, 0.5, 0.2886751, 0.2886751)
    return o.extract(), 4


def test_dense_from_leaves_brute_force():
    lv, D = _small()
    dense = om.dense_from_leaves(lv["keys"], lv["levels"], lv["u"], D)
    x, y, z = morton_decode(lv["keys"])
    s = 1 << (D - lv["levels"].astype(np.int64))
    G = 1 << D
    rng = np.random.default_rng(0)
    for _ in range(200):
        v = rng.integers(0, G, 3)
        hit = [i for i in range(len(s)) if x[i] <= v[0] < x[i] + s[i] and y[i] <= v[1] < y[i] + s[i]
               and z[i] <= v[2] < z[i] + s[i]]
        assert len(hit) == 1
        assert dense[v[2], v[1], v[0]] == np.float32(lv["u"][hit[0]])


def test_vertices_of_a_linear_field_lie_on_its_zero_plane():
    D = 4
    G = 1 << D
    h = 2.0 ** -D
    x0 = 0.37
    xs = (np.arange(G) + 0.5) * h
    dense = np.broadcast_to((xs - x0).astype(np.float32)[None, None, :], (G, G, G)).copy()
    ids, pos = om.crossing_vertices(dense, 0.0, D)
    assert len(ids) == G * G  # one crossing edge per (y, z) row, along x
    assert np.all(ids % 3 == 0)
    assert np.max(np.abs(pos[:, 0] - x0)) < 1e-6
    assert np.all(np.isin(pos[:, 1], ((np.arange(G) + 0.5) * h).astype(np.float32)))


def test_vertices_of_a_sphere_distance_field_are_near_the_sphere():
    D = 5
    G = 1 << D
    c = (np.arange(G) + 0.5) / G
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = 0.31
    dense = (np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) - r).astype(np.float32)
    ids, pos = om.crossing_vertices(dense, 0.0, D)
    d = np.abs(np.linalg.norm(pos - 0.5, axis=1) - r)
    # linear interpolation of a distance field along an edge of length h
    assert d.max() < 0.5 * (1.0 / G) ** 2 / r + 1e-6
    assert len(np.unique(ids)) == len(ids)


def test_quantisation_error_of_fields_built_from_the_leaves():
    lv, D = _small()
    dense = om.dense_from_leaves(lv["keys"], lv["levels"], lv["u"], D)
    assert om.quantisation_error(lv["keys"], lv["levels"], lv["u"], dense, D) == 0.0
    shifted = dense + np.float32(0.25)
    e = om.quantisation_error(lv["keys"], lv["levels"], lv["u"], shifted, D)
    # |u - (u + 0.25)| per leaf, up to the float32 rounding of u + 0.25
    assert abs(e - 0.25 * len(lv["u"])) < 1e-6 * len(lv["u"])


def test_box_forms_agree_with_the_whole_grid():
    """The box forms of the resampling and of the vertex set, used where the
    grid is too large for the whole-grid forms, restrict them exactly: the
    field of a box is that box of the whole field, and the box's vertices are
    the whole grid's vertices whose edge has both voxels in the box."""
    lv, D = _small()
    G = 1 << D
    full = om.dense_from_leaves(lv["keys"], lv["levels"], lv["u"], D)
    ids, pos = om.crossing_vertices(full, 0.0, D)
    assert len(ids) > 50
    vox, axis = ids // 3, ids % 3
    vx, vy, vz = vox % G, (vox // G) % G, vox // (G * G)
    # boxes around two vertices' voxels
    a, b = len(ids) // 3, 2 * len(ids) // 3
    def at(i, back, shape):  # a box inside the grid, from `back` voxels before vertex i's voxel
        return tuple(min(max(0, int(v[i]) - back), G - n) for v, n in zip((vx, vy, vz), shape[::-1]))

    boxes = (((0, 0, 0), (G, G, G)), (at(a, 2, (5, 6, 7)), (5, 6, 7)), (at(b, 1, (7, 4, 5)), (7, 4, 5)))
    for k, (origin, shape) in enumerate(boxes):
        (ox, oy, oz), (nz, ny, nx) = origin, shape
        box = om.dense_box(lv["keys"], lv["levels"], lv["u"], D, origin, shape)
        assert np.array_equal(box, full[oz:oz + nz, oy:oy + ny, ox:ox + nx])
        bi, bp = om.crossing_vertices(box, 0.0, D, origin)
        ex, ey, ez = vx + (axis == 0), vy + (axis == 1), vz + (axis == 2)
        inside = ((vx >= ox) & (ex < ox + nx) & (vy >= oy) & (ey < oy + ny) & (vz >= oz) & (ez < oz + nz))
        assert np.array_equal(bi, ids[inside])
        assert np.array_equal(bp, pos[inside])
        assert k == 0 or 0 < inside.sum() < len(ids)
