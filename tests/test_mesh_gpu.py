"""Meshing and Eq. 7 on the GPU against the evaluation oracle: the
finest-grid field and the marching-cubes vertex set bit for bit, the
triangles checked for validity (they are a choice), Eq. 7 to double
rounding."""
from __future__ import annotations

from collections import Counter

import numpy as np
import pytest

from oracle import Oracle
from oracle import mesh as om
from paper_1608_07411_amd import synth
from tests.helpers import TAU32, base_params, blob_volumes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _fused(D=5, n_views=6, iters=8, noise=0.0, **over):
    w = synth.sphere_workload(max_depth=D, n_views=n_views, W=80, H=60, f=75.0, rel_noise=noise, **over)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    g.fuse(iters, 0.5, TAU32, TAU32)
    return g, D


def _topology(edges):
    tri = [tuple(int(v) for v in t) for t in edges]
    assert all(len(set(t)) == 3 for t in tri), "degenerate triangle"
    und = Counter()
    for a, b, c in tri:
        for e in ((a, b), (b, c), (c, a)):
            und[(min(e), max(e))] += 1
    V = len({v for t in tri for v in t})
    return V, len(und), len(tri), und


def _voxel_of(edge_id, G):
    """(lower voxel (x, y, z), axis) of a grid edge id."""
    v, axis = divmod(int(edge_id), 3)
    return (v % G, (v // G) % G, v // (G * G)), axis


def _components(und):
    parent = {}

    def find(a):
        while parent.setdefault(a, a) != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in und:
        parent[find(a)] = find(b)
    return len({find(a) for e in und for a in e})


def test_dense_field_matches_oracle():
    g, D = _fused()
    lv = g.extract()
    ref = om.dense_from_leaves(lv["keys"], lv["levels"], lv["u"], D)
    assert np.array_equal(g.dense_field(), ref)
    dev = torch.empty((1 << D) ** 3, dtype=torch.float32, device="cuda")
    g.dense_field(dev)
    assert np.array_equal(dev.cpu().numpy().reshape(ref.shape), ref)


# eta = 3 delta at depth 5: with the default 10 delta the band behind the
# surface covers the small domain and no zero level remains
@pytest.mark.parametrize("D,noise,over", [(5, 0.0, dict(eta=0.28125)), (6, 0.005, {})])
def test_mesh_vertices_match_oracle_and_mesh_is_closed(D, noise, over):
    g, D = _fused(D=D, noise=noise, **over)
    xyz, ed = g.mesh(0.0)
    assert len(xyz) > 100
    ids = ed.reshape(-1)
    pts = xyz.reshape(-1, 3)
    uid, first = np.unique(ids, return_index=True)
    # a vertex id always carries the same position
    order = np.argsort(ids, kind="stable")
    same = ids[order][1:] == ids[order][:-1]
    assert np.array_equal(pts[order][1:][same], pts[order][:-1][same])
    ref_ids, ref_pos = om.crossing_vertices(g.dense_field(), 0.0, D)
    assert np.array_equal(uid, ref_ids)
    assert np.array_equal(pts[first], ref_pos)
    V, E, F, und = _topology(ed)
    G = 1 << D
    # every mesh edge is shared by two triangles, except where the surface
    # leaves the grid: then both of its vertices lie on one outermost layer of
    # voxel centres, across that layer's axis
    open_edges = [e for e, k in und.items() if k != 2]
    assert all(und[e] == 1 for e in open_edges)
    for a, b in open_edges:
        ca, cb = _voxel_of(a, G), _voxel_of(b, G)
        assert any(ca[1] != d and cb[1] != d and ca[0][d] == cb[0][d] and ca[0][d] in (0, G - 1)
                   for d in range(3)), f"open mesh edge inside the grid: {ca}, {cb}"
    if not open_edges and noise == 0.0:
        assert V - E + F == 2 * _components(und)  # closed genus-0 pieces


def test_mesh_capacity_protocol_and_iso():
    g, D = _fused(D=5, iters=3, eta=0.28125)
    n0 = g.mesh(0.0)[0].shape[0]
    n1 = g.mesh(0.5)[0].shape[0]
    assert n0 > 0 and n1 > 0 and n0 != n1
    import ctypes as C
    n = C.c_int64(0)
    st = otf.lib().otf_mesh(g.h, C.c_float(0.0), 1, None, None, C.byref(n))
    assert st == 3 and n.value == n0


def test_quantisation_error_matches_oracle():
    g, D = _fused(D=5, iters=10)
    w = synth.sphere_workload(max_depth=5, n_views=6, W=80, H=60, f=75.0, rel_noise=0.0, spread_tau=-1.0,
                              join_tau=2.0)
    dense_ctx = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    dense_ctx.fuse(10, 0.5, TAU32, TAU32)
    ref_field = dense_ctx.dense_field()
    assert dense_ctx.num_leaves() == (1 << D) ** 3  # fully refined, nothing joined
    lv = g.extract()
    e_ref = om.quantisation_error(lv["keys"], lv["levels"], lv["u"], ref_field, D)
    e = g.quantisation_error(ref_field)
    assert abs(e - e_ref) <= 1e-9 * max(1.0, e_ref)
    dev = torch.from_numpy(ref_field).cuda()
    assert g.quantisation_error(dev) == e
    assert g.quantisation_error(g.dense_field()) == 0.0


@pytest.mark.parametrize("D", [3, 5, 7])
def test_eval_on_unbalanced_trees_matches_oracle(D):
    """The field, Eq. 7 and the vertex set on trees built from volumes: one
    chunk of the finest grid holding many leaves (depth 3), several chunks
    (depth 5), and leaves larger than a chunk (depth 7). The field and the
    vertex set bit for bit; Eq. 7 against a random reference field to 1e-9
    (double sums in another order), and exactly 0 against the own field."""
    f, wv = blob_volumes(3, D, seed=D)
    o = Oracle("f32").build_volumes(f, wv, base_params(D))
    g = otf.Context(0).import_state(o.export_state())
    g.fuse(3, 0.5, TAU32, TAU32)
    lv = g.extract()
    if D == 7:
        assert (lv["levels"] < D - 4).any(), "no leaf larger than a chunk"
    ref = om.dense_from_leaves(lv["keys"], lv["levels"], lv["u"], D)
    assert np.array_equal(g.dense_field(), ref)
    rnd = np.random.default_rng(D).standard_normal(ref.shape).astype(np.float32)
    e, e_ref = g.quantisation_error(rnd), om.quantisation_error(lv["keys"], lv["levels"], lv["u"], rnd, D)
    assert abs(e - e_ref) <= 1e-9 * max(1.0, e_ref)
    assert g.quantisation_error(ref) == 0.0
    xyz, ed = g.mesh(0.0)
    uid, first = np.unique(ed.reshape(-1), return_index=True)
    ref_ids, ref_pos = om.crossing_vertices(ref, 0.0, D)
    assert len(ref_ids) > 0
    assert np.array_equal(uid, ref_ids)
    assert np.array_equal(xyz.reshape(-1, 3)[first], ref_pos)
    _topology(ed)


def test_evaluation_kernel_timing():
    """otf_profile_read_eval counts and times the evaluation kernels while
    profiling is on, and otf_profile resets them."""
    g, D = _fused(D=5, iters=3, eta=0.28125)
    g.reset_counters(profile=True)
    field = g.dense_field()
    g.quantisation_error(field)
    g.mesh(0.0)  # the count call, then the call that emits
    k = g.profile_read_eval()
    # the field: once by dense_field, once by each mesh call
    assert {n: v["launches"] for n, v in k.items()} == {"field": 3, "eq7": 1, "mc_count": 2, "mc_emit": 1}
    assert all(v["ms"] > 0 for v in k.values())
    g.reset_counters(profile=False)
    g.dense_field()
    assert all(v["launches"] == 0 for v in g.profile_read_eval().values())


def test_evaluation_at_the_maximum_depth():
    """Depth 10 (1024^3 finest voxels, the deepest octree the library takes):
    the field and the vertex set on sampled 24^3 boxes around mesh vertices
    against the oracle's box forms bit for bit (the triangle count bound of
    this grid exceeds 32 bits, so the per-row counts are summed in 64 bits
    before the offsets), and Eq. 7 exactly 0 against the own field. Splitting
    is off (tau_s = 0): with 4 views much of the domain is unobserved, and the
    split rule would refine it past the 2^26-leaf limit."""
    w = synth.sphere_workload(max_depth=10, n_views=4, split_tau=0.0)
    D = w.max_depth
    G = 1 << D
    g = otf.Context(0).build_octree(torch.from_numpy(w.depth).cuda(), w.cams, w.params)
    g.fuse(2, w.lam, w.tau, w.sigma)
    lv = g.extract()
    field = g.dense_field(torch.empty(G ** 3, dtype=torch.float32, device="cuda")).view(G, G, G)
    xyz, ed = g.mesh(0.0)
    print(f"depth 10: {lv['keys'].size} leaves, {len(xyz)} triangles", flush=True)
    assert len(xyz) > 1000
    ids = ed.reshape(-1)
    pts = xyz.reshape(-1, 3)
    vv, ax = ids // 3, ids % 3
    vx, vy, vz = vv % G, (vv // G) % G, vv // (G * G)
    rng = np.random.default_rng(10)
    n = 24
    for k in rng.choice(ids.size, 3, replace=False):
        origin = tuple(min(max(0, int(a[k]) - n // 2), G - n) for a in (vx, vy, vz))
        ox, oy, oz = origin
        box = om.dense_box(lv["keys"], lv["levels"], lv["u"], D, origin, (n, n, n))
        assert np.array_equal(field[oz:oz + n, oy:oy + n, ox:ox + n].cpu().numpy(), box)
        bid, bpos = om.crossing_vertices(box, 0.0, D, origin)
        inside = ((vx >= ox) & (vx + (ax == 0) < ox + n) & (vy >= oy) & (vy + (ax == 1) < oy + n)
                  & (vz >= oz) & (vz + (ax == 2) < oz + n))
        gid, first = np.unique(ids[inside], return_index=True)
        assert len(bid) > 0
        assert np.array_equal(gid, bid)
        assert np.array_equal(pts[inside][first], bpos)
    assert g.quantisation_error(field.view(-1)) == 0.0
    g.close()
