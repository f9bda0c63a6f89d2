"""Frozen-structure iterations replayed from a recorded HIP graph
(otf_fuse_graph_iterations): bit-identical to the same iterations run one
launch at a time, and to the oracle, with eager work and synchronisations
between the calls that replay the graph."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from paper_1608_07411_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _frozen_sphere():
    w = synth.sphere_workload()  # depth 6, 8 views 160x120
    w.params = dict(w.params, restructure_every=0)
    return w


@pytest.mark.parametrize("solver", ["pd", "gd"])
def test_graph_replay_matches_eager_and_oracle(solver):
    w = _frozen_sphere()
    depth = torch.from_numpy(w.depth).cuda()
    a = otf.Context(0).build_octree(depth, w.cams, w.params)
    b = otf.Context(0).build_octree(depth, w.cams, w.params)
    o = Oracle("f32").import_state(a.export_state())

    def run(ctx, n, eager):
        if solver == "pd":
            if eager:
                for _ in range(n):
                    ctx.fuse(1, w.lam, w.tau, w.sigma)
            else:
                ctx.fuse(n, w.lam, w.tau, w.sigma)
        else:
            if eager:
                for _ in range(n):
                    ctx.fuse_gd(1, 0.5, 0.05, 0.1)
            else:
                ctx.fuse_gd(n, 0.5, 0.05, 0.1)

    # three calls that replay the graph, with eager work (energy, export) and
    # synchronisations between them; each compared with the eager twin
    for n, expect in ((40, 32), (17, 16), (25, 24)):
        run(a, n, eager=False)
        assert a.graph_iterations() == expect
        run(b, n, eager=True)
        assert b.graph_iterations() == 0
        assert a.export_state() == b.export_state(), f"after {n} replayed iterations"
        assert a.energy() == b.energy()
        torch.cuda.synchronize()
    total = 40 + 17 + 25
    if solver == "pd":
        o.fuse(total, w.lam, w.tau, w.sigma)
    else:
        o.fuse_gd(total, 0.5, 0.05, 0.1)
    assert a.export_state() == o.export_state()
    a.close()
    b.close()


def test_short_calls_and_profiling_run_eagerly():
    w = _frozen_sphere()
    a = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    a.fuse(16, w.lam, w.tau, w.sigma)
    assert a.graph_iterations() == 0
    a.reset_counters(profile=True)
    a.fuse(40, w.lam, w.tau, w.sigma)
    assert a.graph_iterations() == 0
    a.reset_counters(profile=False)
    a.fuse(40, w.lam, w.tau, w.sigma)
    assert a.graph_iterations() == 32
    # split/join on: never replayed
    b = otf.Context(0).build_octree(w.depth, w.cams, dict(w.params, restructure_every=1))
    b.fuse(40, w.lam, w.tau, w.sigma)
    assert b.graph_iterations() == 0
    a.close()
    b.close()
