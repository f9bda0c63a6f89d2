"""otf_energy_noalloc, the energy entry point that allocates nothing (its
scratch is a static device array of the library): through the C ABI it must
equal otf_energy bit for bit, on two calls in a row, the second on a smaller
octree, and again on the first after that (nothing stale carries over)."""
from __future__ import annotations

import pytest

from paper_1608_07411_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _ctx(max_depth, n_views, W, H, f):
    w = synth.sphere_workload(max_depth=max_depth, n_views=n_views, W=W, H=H, f=f)
    c = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    c.fuse(5, w.lam, w.tau, w.sigma)
    return c


def test_energy_noalloc_matches_energy():
    big = _ctx(6, 8, 160, 120, 150.0)
    small = _ctx(4, 3, 80, 60, 75.0)
    assert big.num_leaves() > small.num_leaves() > 0
    for c in (big, small, big):
        want = c.energy()
        got = c.energy_noalloc()
        print(f"{c.num_leaves()} leaves: energy {want}, no-alloc {got}", flush=True)
        assert got == want
    big.close()
    small.close()
