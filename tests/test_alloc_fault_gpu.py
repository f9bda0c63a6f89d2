"""Device allocation failures (OTF_E_NOMEM) injected through the
otf_debug_fail_allocations test hook: at every allocation of a build and of
fuse iterations with split/join in turn, the call fails with OTF_E_NOMEM, the
context reports no valid state afterwards (or keeps the built one when only
the fuse failed), it is destroyed cleanly, and the device's free memory
returns to what it was before: nothing leaks."""
from __future__ import annotations

import pytest

from paper_1608_07411_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402

NOMEM, STATE = 2, 5


def _run(w, fail_after):
    """Build and 4 iterations with split/join, the fail_after-th allocation
    failing; returns the step that failed ('build', 'fuse') or None."""
    c = otf.Context(0)
    c.debug_fail_allocations(fail_after)
    failed = None
    try:
        c.build_octree(w.depth, w.cams, w.params)
        try:
            for _ in range(4):
                c.fuse(1, w.lam, w.tau, w.sigma)
        except otf.OtfError as e:
            assert e.status == NOMEM, e
            failed = "fuse"
    except otf.OtfError as e:
        assert e.status == NOMEM, e
        failed = "build"
    if failed:
        with pytest.raises(otf.OtfError) as e:
            c.fuse(1, w.lam, w.tau, w.sigma)
        assert e.value.status == STATE
    c.close()
    return failed


def test_injected_allocation_failures_leave_no_leak():
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0)
    assert _run(w, 0) is None  # warm-up: the runtime's own first-use allocations
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    seen = []
    for k in range(1, 400):
        r = _run(w, k)
        seen.append(r)
        if r is None:
            break
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"allocations failed in turn: {seen.count('build')} during the build, {seen.count('fuse')} during "
          f"the fuse; free memory before {free0}, after {free1}", flush=True)
    assert seen[-1] is None, "more than 400 allocations"
    assert "build" in seen and "fuse" in seen
    assert free1 == free0
