"""Batches (otf_batch): many octrees swept by the same launches.

A batch iteration must equal one otf_fuse iteration of every member alone, bit
for bit (per-leaf arithmetic does not depend on the tiling or launch shape),
through the autotuner's iterations, eager iterations with split/join, and
replays of the captured iteration graph. One member is also checked against
the CPU oracle directly.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from paper_1608_07411_amd import synth
from tests.helpers import TAU32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402

# (max depth, views): octrees of uneven depth and view count
SPECS = [(4, 3), (5, 4), (6, 2), (5, 6), (4, 8)]
LAM = 0.5


def _workloads(restructure_every: int):
    return [synth.sphere_workload(seed=k, max_depth=D, n_views=V, W=80, H=60, f=75.0,
                                  restructure_every=restructure_every) for k, (D, V) in enumerate(SPECS)]


def _pair(ws):
    solo, members = [], []
    for w in ws:
        for out in (solo, members):
            c = otf.Context(0)
            c.build_octree(w.depth, w.cams, w.params)
            out.append(c)
    return solo, members


def _assert_same(solo, members, what):
    for k, (a, b) in enumerate(zip(solo, members)):
        assert a.export_state() == b.export_state(), f"{what}: member {k} differs from its solo run"
        assert a.last_counts() == b.last_counts(), f"{what}: member {k} split/join counts differ"


def test_batch_with_split_join_matches_solo_runs():
    ws = _workloads(restructure_every=1)
    solo, members = _pair(ws)
    batch = otf.Batch(0)
    for m in members:
        batch.add(m)
    for n in (5, 6, 3):  # spans the autotuner's 9 candidate iterations, then eager iterations
        for c in solo:
            c.fuse(n, LAM, TAU32, TAU32)
        batch.fuse(n, LAM, TAU32, TAU32)
        torch.cuda.synchronize()
        _assert_same(solo, members, f"after {n} more iterations")
    cfg = batch.config()
    assert cfg["tuned"] and cfg["block"] in (128, 256, 512)
    batch.close()


def test_batch_member_matches_oracle():
    w = synth.sphere_workload(seed=3, max_depth=5, n_views=4, W=80, H=60, f=75.0)
    ws = [w] + _workloads(restructure_every=1)[:2]
    _, members = _pair(ws)
    batch = otf.Batch(0)
    for m in members:
        batch.add(m)
    o = Oracle("f32").import_state(members[0].export_state())
    batch.fuse(4, LAM, TAU32, TAU32)
    o.fuse(4, LAM, TAU32, TAU32)
    g, r = members[0].extract(), o.extract()
    assert np.array_equal(g["keys"], r["keys"]) and np.array_equal(g["levels"], r["levels"])
    for k in ("u", "ubar"):
        assert np.array_equal(g[k].astype(np.float64), r[k]), k
    assert np.array_equal(g["p"].astype(np.float64), r["p"])


def test_frozen_batch_graph_replays_match_solo_runs():
    ws = _workloads(restructure_every=0)
    solo, members = _pair(ws)
    batch = otf.Batch(0)
    for m in members:
        batch.add(m)
    # 9 tuning iterations, then graph replays (chunks of 16) and an eager rest;
    # eager work and synchronisations between the calls
    for n, graphed in ((9, 0), (40, 32), (16, 16), (7, 0), (33, 32)):
        for c in solo:
            c.fuse(n, LAM, TAU32, TAU32)
        batch.fuse(n, LAM, TAU32, TAU32)
        torch.cuda.synchronize()
        _assert_same(solo, members, f"after {n} more iterations")
        assert batch.config()["graph_iterations"] == graphed
        members[0].energy()  # eager work on a member between replays
    batch.close()


def test_batch_errors():
    ws = _workloads(restructure_every=1)[:2]
    _, members = _pair(ws)
    batch = otf.Batch(0)
    batch.fuse(3, LAM, TAU32, TAU32)  # empty batch: nothing to do
    batch.add(members[0])
    with pytest.raises(otf.OtfError) as e:
        batch.add(members[0])
    assert e.value.status == 1
    other = torch.cuda.Stream()
    c = otf.Context(0, stream=other.cuda_stream)
    c.build_octree(ws[1].depth, ws[1].cams, ws[1].params)
    with pytest.raises(otf.OtfError) as e:
        batch.add(c)
    assert e.value.status == 1
    empty = otf.Context(0)
    with pytest.raises(otf.OtfError) as e:
        batch.add(empty)
    assert e.value.status == 5
    before = members[0].export_state()
    for bad in ((-1, LAM, TAU32, TAU32), (2, -1.0, TAU32, TAU32), (2, LAM, 0.0, TAU32), (2, LAM, TAU32, float("nan"))):
        with pytest.raises(otf.OtfError) as e:
            batch.fuse(*bad)
        assert e.value.status == 1
    assert members[0].export_state() == before
    batch.close()
    torch.cuda.synchronize()
    c.close()


def test_batch_at_object_shapes_matches_solo_runs_and_oracle():
    """The first 12 objects of the 48-object batched workload (spheres of max
    depth 6-9 with 14-59 views 160x120, split/join every iteration): the
    autotuner's 9 iterations and 7 eager ones, every member bit for bit
    against its solo run; the depth-6 member also against the fp32 oracle.
    Some members' adjacency has lists longer than 64 entries (the long-list
    waves run)."""
    ws = synth.batch_workloads(12, restructure_every=1)
    depths = sorted({w.max_depth for w in ws})
    assert depths == [6, 7, 8, 9]
    solo, members = _pair(ws)
    k6 = next(k for k, w in enumerate(ws) if w.max_depth == 6)
    o = Oracle("f32").import_state(members[k6].export_state())
    n_long = 0
    for c in members:
        counts, _ = c.extract_neighbours()
        n_long += int(np.count_nonzero((counts[:, :3].sum(1) > 64) | (counts[:, 3:].sum(1) > 64)))
    assert n_long > 0
    batch = otf.Batch(0)
    for m in members:
        batch.add(m)
    for n in (9, 7):
        for c in solo:
            c.fuse(n, LAM, TAU32, TAU32)
        batch.fuse(n, LAM, TAU32, TAU32)
        o.fuse(n, LAM, TAU32, TAU32)
        torch.cuda.synchronize()
        _assert_same(solo, members, f"after {n} more iterations")
        assert members[k6].export_state() == o.export_state(), "depth-6 member differs from the oracle"
    assert batch.config()["tuned"]
    batch.close()


def test_batch_members_refuse_solo_calls_and_leave_when_destroyed():
    ws = _workloads(restructure_every=1)[:3]
    solo, members = _pair(ws)
    batch = otf.Batch(0)
    for m in members:
        batch.add(m)
    blob = members[0].export_state()
    w = ws[0]
    for call in (lambda c: c.fuse(1, LAM, TAU32, TAU32), lambda c: c.fuse_gd(1, 0.5, 0.05, 0.3),
                 lambda c: c.build_octree(w.depth, w.cams, w.params), lambda c: c.import_state(blob)):
        with pytest.raises(otf.OtfError) as e:
            call(members[0])
        assert e.value.status == 5 and "batch member" in str(e.value)
    assert members[0].export_state() == blob
    # a destroyed member leaves the batch; the others go on as before
    members[1].close()
    batch.fuse(3, LAM, TAU32, TAU32)
    for k in (0, 2):
        solo[k].fuse(3, LAM, TAU32, TAU32)
    torch.cuda.synchronize()
    for k in (0, 2):
        assert members[k].export_state() == solo[k].export_state()
    batch.close()
    members[0].fuse(1, LAM, TAU32, TAU32)  # free again once the batch is gone
