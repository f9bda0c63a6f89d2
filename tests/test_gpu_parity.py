"""Parity of the HIP path (through the C ABI) with the CPU oracle.

The oracle runs in its canonical fp32 mode, whose operation order the kernels
follow, so structure, observations and values are compared bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_1608_07411_amd import synth
from tests.helpers import TAU32, base_params, blob_set, blob_set_leaves, blob_volumes, parse_views, plane_volumes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _ctx():
    return otf.Context(0)


def _same_leaves(g: dict, o: dict, what=""):
    assert np.array_equal(g["keys"], o["keys"]), f"{what}: keys differ"
    assert np.array_equal(g["levels"], o["levels"]), f"{what}: levels differ"
    for k in ("u", "ubar"):
        a, b = g[k].astype(np.float64), o[k]
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{what}: {k} differs at {bad[:5]} gpu={a[bad[:5]]} oracle={b[bad[:5]]}"
    a, b = g["p"].astype(np.float64), o["p"]
    assert np.array_equal(a, b), f"{what}: p differs"


def _small_sphere(**kw):
    return synth.sphere_workload(max_depth=kw.pop("max_depth", 5), n_views=kw.pop("n_views", 4), W=80, H=60,
                                 f=75.0, **kw)


def test_build_blob_identical():
    w = _small_sphere()
    g = _ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    gb, ob = g.export_state(), o.export_state()
    gv, gl = parse_views(gb)
    ov, ol = parse_views(ob)
    for v in range(len(ov)):
        assert np.array_equal(gv[v], ov[v]), f"view {v} octree differs"
    assert np.array_equal(gl, ol)
    assert gb == ob


def test_build_from_device_depth_identical():
    w = _small_sphere(n_views=3)
    dev = torch.from_numpy(w.depth).cuda()
    g = _ctx().build_octree(dev, w.cams, w.params)
    h = _ctx().build_octree(w.depth, w.cams, w.params)
    assert g.export_state() == h.export_state()


def test_observations_and_adjacency_identical():
    w = _small_sphere()
    g = _ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    go, oo = g.extract_obs(), o.leaf_obs()
    assert np.array_equal(go["M"], oo["M"])
    for k in ("F", "W", "wtot", "inv"):
        assert np.array_equal(go[k].astype(np.float64), oo[k]), k
    gc, gi = g.extract_neighbours()
    oc, oi = o.neighbours()
    assert np.array_equal(gc, oc)
    assert np.array_equal(gi, oi)


def test_adjacency_and_observations_after_restructuring():
    """Incrementally rebuilt adjacency and appended observations equal the
    oracle's from-scratch ones after many split/join steps."""
    w = _small_sphere()
    g = _ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    changed = 0
    for _ in range(8):
        g.fuse(2, w.lam, w.tau, w.sigma)
        o.fuse(2, w.lam, w.tau, w.sigma)
        changed += sum(o.last_counts())
        gc, gi = g.extract_neighbours()
        oc, oi = o.neighbours()
        assert np.array_equal(gc, oc) and np.array_equal(gi, oi)
        go, oo = g.extract_obs(), o.leaf_obs()
        assert np.array_equal(go["M"], oo["M"])
        for k in ("F", "W", "wtot", "inv"):
            assert np.array_equal(go[k].astype(np.float64), oo[k]), k
    assert changed > 0


def test_observation_pool_compaction_parity():
    """Restructures append new leaves' observations to the pool and compact it
    in leaf order when it fills: the observations stay identical to the
    oracle's through at least one compaction."""
    w = _small_sphere()
    g = _ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    for _ in range(40):
        g.fuse(1, w.lam, w.tau, w.sigma)
        o.fuse(1, w.lam, w.tau, w.sigma)
        go, oo = g.extract_obs(), o.leaf_obs()
        assert np.array_equal(go["M"], oo["M"])
        for k in ("F", "W", "wtot", "inv"):
            assert np.array_equal(go[k].astype(np.float64), oo[k]), k
        st = g.obs_pool_stats()
        assert st["used"] <= st["capacity"]
        if st["compactions"] >= 2:
            break
    assert g.obs_pool_stats()["compactions"] >= 1
    _same_leaves(g.extract(), o.extract(), "after the compactions")


@pytest.mark.parametrize("restructure", [0, 1])
def test_free_running_parity_small(restructure):
    w = _small_sphere()
    prm = dict(w.params, restructure_every=restructure)
    g = _ctx().build_octree(w.depth, w.cams, prm)
    o = Oracle("f32").build(w.depth, w.cams, prm)
    for step in range(6):
        g.fuse(5, w.lam, w.tau, w.sigma)
        o.fuse(5, w.lam, w.tau, w.sigma)
        _same_leaves(g.extract(), o.extract(), f"after {5 * (step + 1)} iterations")
        assert g.last_counts() == o.last_counts()


def test_same_state_single_step_from_oracle_blob():
    w = _small_sphere(n_views=3)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    o.fuse(3, w.lam, w.tau, w.sigma)
    blob = o.export_state()
    g = _ctx().import_state(blob)
    assert g.export_state() == blob
    o.fuse(1, w.lam, w.tau, w.sigma)
    g.fuse(1, w.lam, w.tau, w.sigma)
    assert g.last_counts() == o.last_counts()
    assert g.export_state() == o.export_state()


@pytest.mark.parametrize("maker,D,seed", [(plane_volumes, 4, 1), (blob_volumes, 5, 4), (blob_volumes, 5, 8)])
def test_volume_states_parity(maker, D, seed):
    f, w = maker(3, D, seed, p_unobs=0.2)
    o = Oracle("f32").build_volumes(f, w, base_params(D))
    g = _ctx().import_state(o.export_state())
    for _ in range(4):
        o.fuse(3, 0.5, TAU32, TAU32)
        g.fuse(3, 0.5, TAU32, TAU32)
        assert g.export_state() == o.export_state()


def test_fully_refined_fixed_structure_parity():
    D = 4
    rng = np.random.default_rng(3)
    G = 1 << D
    f = rng.uniform(-1, 1, (4, G, G, G)).astype(np.float32)
    w = (rng.uniform(size=(4, G, G, G)) > 0.3).astype(np.uint8)
    w[0] = 1
    prm = base_params(D, spread_tau=-1.0, split_tau=0.0, join_tau=2.0, restructure_every=0)
    o = Oracle("f32").build_volumes(f, w, prm)
    assert o.num_leaves() == G ** 3
    g = _ctx().import_state(o.export_state())
    o.fuse(40, 0.5, TAU32, TAU32)
    g.fuse(40, 0.5, TAU32, TAU32)
    _same_leaves(g.extract(), o.extract(), "fully refined")


def test_sphere_workload_full_parity():
    """The 64^3, 8-view sphere workload: 200 iterations with split and join."""
    w = synth.workload(1)
    g = _ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    assert g.export_state() == o.export_state()
    for k in range(4):
        g.fuse(50, w.lam, w.tau, w.sigma)
        o.fuse(50, w.lam, w.tau, w.sigma)
        _same_leaves(g.extract(), o.extract(), f"sphere after {50 * (k + 1)}")


def test_energy_matches_oracle():
    w = _small_sphere()
    g = _ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    g.fuse(7, w.lam, w.tau, w.sigma)
    o.fuse(7, w.lam, w.tau, w.sigma)
    gt, gd = g.energy()
    ot, od = o.energy()
    assert abs(gt - ot) <= 1e-10 * abs(ot)
    assert abs(gd - od) <= 1e-10 * abs(od)


def test_lambda_infinity_single_view_gpu():
    w = synth.sphere_workload(max_depth=5, n_views=1, W=80, H=60, f=75.0)
    prm = dict(w.params, restructure_every=2)
    g = _ctx().build_octree(w.depth, w.cams, prm)
    g.fuse(7, 1e30, TAU32, TAU32)
    ex = g.extract()
    ob = g.extract_obs()
    obs = ob["M"] == 1
    assert obs.sum() > 100
    assert np.array_equal(ex["u"][obs], ob["F"][ob["off"][:-1][obs]])


def test_determinism_two_runs():
    w = _small_sphere()
    a = _ctx().build_octree(w.depth, w.cams, w.params).fuse(20, w.lam, w.tau, w.sigma)
    b = _ctx().build_octree(w.depth, w.cams, w.params).fuse(20, w.lam, w.tau, w.sigma)
    assert a.export_state() == b.export_state()


def test_thresholds_disable_split_and_join_gpu():
    w = _small_sphere()
    g = _ctx().build_octree(w.depth, w.cams, dict(w.params, split_tau=0.0))
    n0 = g.num_leaves()
    for _ in range(5):
        g.fuse(1, w.lam, w.tau, w.sigma)
        assert g.last_counts()[0] == 0
    assert g.num_leaves() <= n0
    g = _ctx().build_octree(w.depth, w.cams, dict(w.params, join_tau=1.5))
    for _ in range(5):
        g.fuse(1, w.lam, w.tau, w.sigma)
        assert g.last_counts()[1] == 0


def test_error_paths():
    w = _small_sphere(n_views=2)
    g = _ctx()
    with pytest.raises(otf.OtfError) as e:
        g.fuse(1, 0.5, TAU32, TAU32)
    assert e.value.status == 5  # no state yet
    with pytest.raises(otf.OtfError) as e:
        g.build_octree(w.depth, w.cams, dict(w.params, split_tau=0.95, join_tau=0.9))
    assert e.value.status == 1
    g.build_octree(w.depth, w.cams, w.params)
    for bad in ((float("nan"), TAU32, TAU32), (0.5, 0.0, TAU32), (-1.0, TAU32, TAU32), (0.5, TAU32, float("inf"))):
        with pytest.raises(otf.OtfError) as e:
            g.fuse(1, *bad)
        assert e.value.status == 1
    g.fuse(1, 0.5, TAU32, TAU32)  # state is still valid after rejected arguments
    # capacity: a leaf cap at the initial count, below what the first splits need
    n0 = _ctx().build_octree(w.depth, w.cams, w.params).num_leaves()
    h = _ctx().build_octree(w.depth, w.cams, dict(w.params, max_leaves=n0))
    with pytest.raises(otf.OtfError) as e:
        h.fuse(3, 0.5, TAU32, TAU32)
    assert e.value.status == 3
    with pytest.raises(otf.OtfError) as e:
        h.extract()
    assert e.value.status == 5
    # a corrupt blob is rejected before any device work
    blob = bytearray(g.export_state())
    blob[0] = ord("X")
    with pytest.raises(otf.OtfError) as e:
        _ctx().import_state(bytes(blob))
    assert e.value.status == 1


def _slab_volumes(D, x0, width=2, seed=0):
    G = 1 << D
    rng = np.random.default_rng(seed)
    f = np.ones((2, G, G, G), np.float32)
    f[:, :, :, x0:x0 + width] = rng.uniform(-1, 1, (2, G, G, width)).astype(np.float32)
    return f, np.ones((2, G, G, G), np.uint8)


@pytest.mark.parametrize("D,x0", [(6, 32), (6, 30), (7, 64), (7, 62), (8, 128), (8, 126)])
def test_long_adjacency_lists_parity(D, x0):
    """Half-domain leaves against a refined slab: + lists (slab right of the
    middle) or - lists (left of it) of 32^2 entries (one LDS chunk), 64^2 or
    128^2 (several chunks) are summed in the canonical order."""
    f, w = _slab_volumes(D, x0)
    o = Oracle("f32").build_volumes(f, w, base_params(D))
    counts, _ = o.neighbours()
    side = 1 << (D - 1)
    col = slice(0, 3) if x0 >= side else slice(3, 6)
    assert counts[:, col].sum(1).max() >= side * side
    g = _ctx().import_state(o.export_state())
    for _ in range(3):
        o.fuse(2, 0.5, TAU32, TAU32)
        g.fuse(2, 0.5, TAU32, TAU32)
        assert g.export_state() == o.export_state()


# ---------------------------------------------------------------- edge cases
def _run_both(w, prm, steps, chunk):
    g = _ctx().build_octree(w.depth, w.cams, prm)
    o = Oracle("f32").build(w.depth, w.cams, prm)
    assert g.export_state() == o.export_state(), "built states differ"
    done = 0
    while done < steps:
        g.fuse(chunk, w.lam, w.tau, w.sigma)
        o.fuse(chunk, w.lam, w.tau, w.sigma)
        done += chunk
        _same_leaves(g.extract(), o.extract(), f"after {done} iterations")
        assert g.last_counts() == o.last_counts()
    assert g.export_state() == o.export_state()
    return g, o


def test_no_observations_parity():
    """Every range-map pixel invalid: no leaf has an observation and every
    view octree is its root, so the fused octree starts as one leaf with
    u = 0; |u| < tau_s flags it to split, and the split cascade refines the
    whole domain to the maximum depth, where u stays 0 (a degenerate case of
    the split rule) and no join applies."""
    w = _small_sphere()
    w.depth[:] = 0.0
    g, o = _run_both(w, w.params, 10, 5)
    e = g.extract()
    assert len(e["keys"]) == 8 ** w.max_depth and np.all(e["u"] == 0.0)
    assert g.energy() == (0.0, 0.0)



@pytest.mark.parametrize("lam_scale", [0.0, 1.0])
def test_subnormal_values_parity(lam_scale):
    """Leaf values in the fp32 subnormal range (integers times 2^-140) go through
    the sweep unflushed: bit-identical to the oracle, and with lambda = 0 every
    u and nearly every p is still a nonzero subnormal afterwards. With the
    workload's lambda every leaf here is observed, so the first prox steps
    start from subnormal u and end at range values."""
    w = _small_sphere(restructure_every=0)
    blob = Oracle("f32").build(w.depth, w.cams, w.params).export_state()
    n = len(Oracle("f32").import_state(blob).extract()["u"])
    u = (np.random.default_rng(1).integers(-1000, 1001, n) * 2.0 ** -140).astype(np.float32)
    blob = blob_set_leaves(blob, u=u, ubar=u, p=np.zeros((n, 3), np.float32))
    g, o = _ctx().import_state(blob), Oracle("f32").import_state(blob)
    lam = lam_scale * w.lam
    for done in (3, 6):
        g.fuse(3, lam, w.tau, w.sigma)
        o.fuse(3, lam, w.tau, w.sigma)
        _same_leaves(g.extract(), o.extract(), f"after {done} iterations")
    e = g.extract()
    tiny = np.finfo(np.float32).tiny
    sub_u = (e["u"] != 0) & (np.abs(e["u"]) < tiny)
    sub_p = (e["p"] != 0) & (np.abs(e["p"]) < tiny)
    if lam_scale == 0.0:
        assert sub_u.all() and sub_p.mean() > 0.99
    assert g.export_state() == o.export_state()


@pytest.mark.parametrize("n_views", [32, 33])
def test_prox_wave_segment_boundary_parity(n_views):
    """Leaves of 23 to 32 observations (32 views: every wave takes the prox of
    two leaves per step on half-waves, up to all 32 lanes of a half) and up to
    33 (33 views: a wave holding a leaf of 33 observations takes whole waves,
    the others half-waves): bit-identical to the oracle through iterations
    with split/join."""
    f, wv = blob_volumes(n_views, 4, seed=n_views, p_unobs=0.1)
    o = Oracle("f32").build_volumes(f, wv, base_params(4))
    M = o.leaf_obs()["M"]
    assert M.max() == n_views and M.min() < 32
    g = _ctx().import_state(o.export_state())
    for done in (5, 10):
        g.fuse(5, 0.5, TAU32, TAU32)
        o.fuse(5, 0.5, TAU32, TAU32)
        _same_leaves(g.extract(), o.extract(), f"after {done} iterations")
        assert g.last_counts() == o.last_counts()
    assert g.export_state() == o.export_state()

@pytest.mark.parametrize("n_views", [1, 64])
def test_view_count_extremes_parity(n_views):
    """One view and the 64-view maximum (the fetch's segment of 64 lanes, one
    per view), on small range maps: build, then iterations with split/join.
    The solid band is 3 delta: at depth 5 the workload's 10 delta spans the
    whole domain, and with many views every leaf then starts solid."""
    w = synth.sphere_workload(max_depth=5, n_views=n_views, W=64, H=48, f=60.0)
    prm = dict(w.params, eta=3 * w.params["delta"])
    g, _ = _run_both(w, prm, 20, 5)
    u = g.extract()["u"]
    assert (u < 0).any() and (u > 0).any()


@pytest.mark.parametrize("max_depth", [1, 2, 3])
def test_tiny_trees_parity(max_depth):
    """The smallest trees (2^3 to 8^3 finest voxels): leaves at the domain
    boundary on most faces, lists of one or two entries, splits capped at the
    maximum depth right away."""
    w = synth.sphere_workload(max_depth=max_depth, n_views=4, W=32, H=24, f=30.0)
    _run_both(w, w.params, 12, 4)


def test_build_argument_limits():
    """Arguments outside the documented limits are rejected before any device
    work (OTF_E_INVALID), and the context stays usable."""
    w = _small_sphere(n_views=2)
    g = _ctx()
    bad_params = [dict(max_depth=0), dict(max_depth=11), dict(gamma=0.0), dict(gamma=-1.0),
                  dict(eta=0.5 * w.params["delta"]), dict(delta=0.0), dict(split_tau=0.95, join_tau=0.9)]
    for over in bad_params:
        with pytest.raises(otf.OtfError) as e:
            g.build_octree(w.depth, w.cams, dict(w.params, **over))
        assert e.value.status == 1, over
    for n in (0, 65):
        depth = np.zeros((n, w.depth.shape[1], w.depth.shape[2]), np.float32)
        cams = np.resize(w.cams, n) if n else w.cams[:0]
        with pytest.raises(otf.OtfError) as e:
            g.build_octree(depth, cams, w.params)
        assert e.value.status == 1, n
    g.build_octree(w.depth, w.cams, w.params)
    with pytest.raises(otf.OtfError) as e:
        g.fuse(-1, w.lam, w.tau, w.sigma)
    assert e.value.status == 1
    g.fuse(0, w.lam, w.tau, w.sigma)  # zero iterations: nothing happens
    g.fuse(2, w.lam, w.tau, w.sigma)
