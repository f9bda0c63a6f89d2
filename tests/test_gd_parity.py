"""Parity of the paper's gradient-descent solver (otf_fuse_gd) with the CPU
oracle in its canonical fp32 mode: structure, values and split/join counts
bit for bit, and the smoothed energy terms to double rounding."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from paper_1608_07411_amd import synth
from tests.helpers import base_params, blob_set, blob_volumes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _same(g, o, what):
    assert np.array_equal(g["keys"], o["keys"]), f"{what}: keys"
    assert np.array_equal(g["levels"], o["levels"]), f"{what}: levels"
    for k in ("u", "ubar"):
        a, b = g[k].astype(np.float64), o[k]
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{what}: {k} at {bad[:5]} gpu={a[bad[:5]]} oracle={b[bad[:5]]}"
    assert np.array_equal(g["p"].astype(np.float64), o["p"]), f"{what}: p"


@pytest.mark.parametrize("lam,step,eps", [(0.5, 0.05, 0.3), (1.0, 0.1, 0.5)])
def test_gd_free_running_with_split_join(lam, step, eps):
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    splits = joins = 0
    for it in range(12):
        g.fuse_gd(1, lam, step, eps)
        o.fuse_gd(1, lam, step, eps)
        assert g.last_counts() == o.last_counts(), f"iteration {it}: split/join counts"
        s, j = o.last_counts()
        splits, joins = splits + s, joins + j
        if it % 4 == 3:
            _same(g.extract(), o.extract(), f"iteration {it}")
    assert splits > 0 and joins > 0  # the cascade and the collapse both ran
    tg, dg = g.energy_eps(eps)
    to, do = o.energy_eps(eps)
    assert abs(tg - to) <= 1e-9 * abs(to) and abs(dg - do) <= 1e-9 * abs(do)


def test_gd_paper_schedule_on_volume_state():
    """Unbalanced tree from per-voxel volumes; the paper's step schedule (0.1,
    halved every 20 steps) for 40 steps."""
    f, w = blob_volumes(3, 5, 7, p_unobs=0.1)
    o = Oracle("f32").build_volumes(f, w, base_params(5))
    g = otf.Context(0).import_state(o.export_state())
    step = 0.1
    for k in range(2):
        g.fuse_gd(20, 0.5, step, 0.3)
        o.fuse_gd(20, 0.5, step, 0.3)
        _same(g.extract(), o.extract(), f"after {20 * (k + 1)} steps")
        step *= 0.5


def test_gd_then_primal_dual_on_the_same_context():
    """Switching solvers on one context: each call uses its own solver for the
    split children (the state carries no solver)."""
    w = synth.sphere_workload(max_depth=5, n_views=3, W=80, H=60, f=75.0)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    tau = float(np.float32(1.0 / np.sqrt(12.0)))
    for ctx in (g, o):
        ctx.fuse_gd(5, 0.5, 0.05, 0.3)
        ctx.fuse(5, 0.5, tau, tau)
        ctx.fuse_gd(3, 0.5, 0.05, 0.3)
    _same(g.extract(), o.extract(), "gd, pd, gd")


def test_gd_invalid_arguments():
    w = synth.sphere_workload(max_depth=4, n_views=2, W=80, H=60, f=75.0)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    before = g.export_state()
    for bad in ((-1, 0.5, 0.1, 0.1), (1, -0.5, 0.1, 0.1), (1, 0.5, 0.0, 0.1), (1, 0.5, 0.1, 0.0),
                (1, float("inf"), 0.1, 0.1)):
        with pytest.raises(otf.OtfError) as e:
            g.fuse_gd(*bad)
        assert e.value.status == 1
    assert g.export_state() == before
    with pytest.raises(otf.OtfError):
        g.energy_eps(0.0)
    empty = otf.Context(0)
    with pytest.raises(otf.OtfError) as e:
        empty.fuse_gd(1, 0.5, 0.1, 0.1)
    assert e.value.status == 5


@pytest.mark.parametrize("D,x0", [(6, 32), (6, 30), (7, 62)])
def test_gd_long_adjacency_lists_parity(D, x0):
    """Gradient descent on half-domain leaves against a refined slab: the flux
    sweep's long + lists and the update's long - lists (thousands of entries,
    several chunks) in the canonical sequential order."""
    G = 1 << D
    rng = np.random.default_rng(1)
    f = np.ones((2, G, G, G), np.float32)
    f[:, :, :, x0:x0 + 2] = rng.uniform(-1, 1, (2, G, G, 2)).astype(np.float32)
    w = np.ones((2, G, G, G), np.uint8)
    o = Oracle("f32").build_volumes(f, w, base_params(D))
    counts, _ = o.neighbours()
    assert max(counts[:, :3].sum(1).max(), counts[:, 3:].sum(1).max()) > 64
    g = otf.Context(0).import_state(o.export_state())
    for k in range(3):
        g.fuse_gd(2, 0.5, 0.05, 0.3)
        o.fuse_gd(2, 0.5, 0.05, 0.3)
        assert g.export_state() == o.export_state(), f"after {2 * (k + 1)} steps"
