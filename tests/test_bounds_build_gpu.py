"""The bounds-checked build (libotf_bounds.so, OTF_DEBUG_BOUNDS): the sweeps
check every adjacency range, neighbour index, level code and observation
index they read; every device buffer is followed by a guard zone checked when
the buffer is freed and after every call; every adjacency slot is checked
after each neighbour search (written, neighbour index and level in range). On
valid states it must report nothing and give the same results as the oracle
bit for bit (sphere workload with split/join, long adjacency lists); an entry
pointed past the last leaf from the host (a test hook of that build only) must
be reported as OTF_E_DEVICE, with the bad read sent to index 0 so that every
kernel still ends normally, and so must a guard byte changed from the host
and an adjacency slot left as no search had written it. The default build
refuses the hooks."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from paper_1608_07411_amd import synth
from tests.helpers import TAU32, base_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _bounds_ctx():
    return otf.Context(0, library=otf.BOUNDS_LIB_PATH)


def test_bounds_build_reports_nothing_and_matches_oracle():
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0)
    g = _bounds_ctx().build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    for _ in range(3):
        g.fuse(10, w.lam, w.tau, w.sigma)
        o.fuse(10, w.lam, w.tau, w.sigma)
        assert g.export_state() == o.export_state()
    g.fuse_gd(5, 0.5, 0.05, 0.3)
    o.fuse_gd(5, 0.5, 0.05, 0.3)
    assert g.export_state() == o.export_state()
    g.close()
    # long lists (thousands of entries): the long-list waves' reads
    D, G = 6, 64
    rng = np.random.default_rng(0)
    f = np.ones((2, G, G, G), np.float32)
    f[:, :, :, 32:34] = rng.uniform(-1, 1, (2, G, G, 2)).astype(np.float32)
    o = Oracle("f32").build_volumes(f, np.ones((2, G, G, G), np.uint8), base_params(D))
    g = _bounds_ctx().import_state(o.export_state())
    g.fuse(4, 0.5, TAU32, TAU32)
    o.fuse(4, 0.5, TAU32, TAU32)
    assert g.export_state() == o.export_state()
    g.close()


def test_bounds_build_at_the_timed_workload_size():
    """The depth-9 workload (~1.3e7 leaves, 64 range maps 640x480, lists up to
    thousands of entries) for 6 iterations with split/join under the checked
    build: no index is reported, and the state equals the default build's."""
    w = synth.thin_workload(seed=0)
    depth = torch.from_numpy(w.depth).cuda()
    g = _bounds_ctx().build_octree(depth, w.cams, w.params)
    d = otf.Context(0).build_octree(depth, w.cams, w.params)
    for _ in range(2):
        g.fuse(3, w.lam, w.tau, w.sigma)
        d.fuse(3, w.lam, w.tau, w.sigma)
        assert g.num_leaves() == d.num_leaves() and g.last_counts() == d.last_counts()
    assert g.export_state() == d.export_state()
    g.close()
    d.close()


def test_bounds_build_at_the_maximum_depth():
    """Depth 10, the deepest octree the library takes (30-bit keys, the
    coupling tables' deepest levels; splitting off, since with 4 views the
    split rule would refine the unobserved space past the leaf limit): 4
    iterations with joins and the paper's gradient descent for 2 under the
    checked build report no index and give the default build's state."""
    w = synth.sphere_workload(max_depth=10, n_views=4, split_tau=0.0)
    depth = torch.from_numpy(w.depth).cuda()
    g = _bounds_ctx().build_octree(depth, w.cams, w.params)
    d = otf.Context(0).build_octree(depth, w.cams, w.params)
    for c in (g, d):
        c.fuse(4, w.lam, w.tau, w.sigma)
        c.fuse_gd(2, 0.5, 0.05, 0.3)
    print(f"depth 10: {d.num_leaves()} leaves, last split/join {d.last_counts()}", flush=True)
    assert g.num_leaves() == d.num_leaves()
    assert g.export_state() == d.export_state()
    g.close()
    d.close()


def test_bounds_build_reports_a_bad_index():
    # no restructuring: only the sweeps (which check and redirect) read the
    # corrupted entry
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0, restructure_every=0)
    g = _bounds_ctx().build_octree(w.depth, w.cams, w.params)
    g.fuse(2, w.lam, w.tau, w.sigma)
    counts, _ = g.extract_neighbours()
    leaf = int(np.nonzero(counts[:, :3].sum(1) > 0)[0][0])
    g.debug_corrupt_adjacency(leaf)
    with pytest.raises(otf.OtfError) as e:
        g.fuse(1, w.lam, w.tau, w.sigma)
    assert e.value.status == 4 and "bounds-checked" in str(e.value)
    g.close()
    # the default build refuses the hook and keeps its state
    d = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    before = d.export_state()
    with pytest.raises(otf.OtfError) as e:
        d.debug_corrupt_adjacency(leaf)
    assert e.value.status == 1
    assert d.export_state() == before
    d.close()


def test_bounds_build_reports_a_damaged_guard_zone():
    """One byte changed from the host in the guard zone after the + adjacency
    list: the next call fails with OTF_E_DEVICE and names the place that
    reserved the list; the default build refuses the hook."""
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0, restructure_every=0)
    g = _bounds_ctx().build_octree(w.depth, w.cams, w.params)
    g.fuse(1, w.lam, w.tau, w.sigma)
    g.debug_poke_guard()
    with pytest.raises(otf.OtfError) as e:
        g.fuse(1, w.lam, w.tau, w.sigma)
    assert e.value.status == 4
    assert "past the end of a device buffer" in str(e.value) and "nbr.hip" in str(e.value)
    g.close()
    # the zone was reported once: a new context on the checked build runs clean
    h = _bounds_ctx().build_octree(w.depth, w.cams, w.params)
    h.fuse(2, w.lam, w.tau, w.sigma)
    h.close()
    d = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    with pytest.raises(otf.OtfError) as e:
        d.debug_poke_guard()
    assert e.value.status == 1
    d.close()


def test_bounds_build_reports_an_unwritten_adjacency_slot():
    """The next neighbour search (the restructure of the next solver call)
    leaves + slot 0 unwritten: its adjacency check fails that call with
    OTF_E_DEVICE before any sweep reads the slot; the default build refuses
    the hook."""
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0)
    g = _bounds_ctx().build_octree(w.depth, w.cams, w.params)
    g.fuse(1, w.lam, w.tau, w.sigma)
    g.debug_unwritten_slot()
    with pytest.raises(otf.OtfError) as e:
        for _ in range(20):  # until a restructure searches again
            g.fuse(1, w.lam, w.tau, w.sigma)
    assert e.value.status == 4
    assert "adjacency check" in str(e.value) and "written by no search" in str(e.value)
    g.close()
    d = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    with pytest.raises(otf.OtfError) as e:
        d.debug_unwritten_slot()
    assert e.value.status == 1
    d.close()


def test_bounds_build_batch_reports_nothing_and_matches_solo_runs():
    """The batched sweeps under the checked build (members of uneven depth,
    split/join every iteration, through the autotuner's iterations and eager
    ones; then frozen members through graph replays): no index is reported,
    no guard zone or adjacency slot is bad, and every member equals its solo
    run on the default build."""
    from tests.helpers import TAU32
    for every, steps in ((1, (5, 6, 3)), (0, (9, 40))):
        ws = [synth.sphere_workload(seed=k, max_depth=D, n_views=V, W=80, H=60, f=75.0, restructure_every=every)
              for k, (D, V) in enumerate([(4, 3), (5, 4), (6, 2)])]
        solo = [otf.Context(0).build_octree(w.depth, w.cams, w.params) for w in ws]
        members = [_bounds_ctx().build_octree(w.depth, w.cams, w.params) for w in ws]
        batch = otf.Batch(0, library=otf.BOUNDS_LIB_PATH)
        for m in members:
            batch.add(m)
        for n in steps:
            for c in solo:
                c.fuse(n, 0.5, TAU32, TAU32)
            batch.fuse(n, 0.5, TAU32, TAU32)
            for a, b in zip(solo, members):
                assert a.export_state() == b.export_state() and a.last_counts() == b.last_counts()
        if every == 0:
            assert batch.config()["graph_iterations"] > 0
        batch.close()
        for c in solo + members:
            c.close()
