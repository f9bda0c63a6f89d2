"""Oracle parity on the plain-method workloads at their full sizes, through
the C ABI.

* Depth-8 blocks workload (6 spheres and 4 oriented boxes, 32 range maps
  640x480, one-voxel noise and 2% outlier pixels, split/join every
  iteration): the build and 50 free-running iterations against the canonical
  fp32 oracle, the state blob bit for bit every 10 iterations and the split
  and join counts of every iteration. The module's tests share the two
  solvers and run in order, 10 iterations each.
* Depth-6 sphere workload (8 range maps 160x120): 200 iterations with
  split/join on the GPU (fp32) against the oracle in fp64 from the same
  start. The converged result must keep the same structure, the energy of
  Eq. 3 with the normaliser of Eq. 5 within 1e-6 relative, and u resampled
  to the finest grid within 1e-5 everywhere.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from paper_1608_07411_amd import synth
from tests.helpers import to_dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


@pytest.fixture(scope="module")
def blocks():
    w = synth.workload(2)
    print("blocks workload: depth 8, 32 views 640x480", flush=True)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    o = Oracle("f32").build(w.depth, w.cams, w.params)
    state = dict(w=w, g=g, o=o, done=0)
    yield state
    g.close()


def test_blocks_build_identical(blocks):
    g, o = blocks["g"], blocks["o"]
    assert g.num_leaves() > 3_000_000
    assert g.export_state() == o.export_state()


@pytest.mark.parametrize("chunk", range(5))
def test_blocks_free_running_parity(blocks, chunk):
    w, g, o = blocks["w"], blocks["g"], blocks["o"]
    assert blocks["done"] == 10 * chunk, "chunks run in order"
    for it in range(10):
        g.fuse(1, w.lam, w.tau, w.sigma)
        o.fuse(1, w.lam, w.tau, w.sigma)
        assert g.last_counts() == o.last_counts(), f"iteration {blocks['done'] + it + 1}: split/join counts"
    blocks["done"] += 10
    assert g.export_state() == o.export_state(), f"state after {blocks['done']} iterations"
    print(f"blocks: {blocks['done']} iterations identical, {g.num_leaves()} leaves", flush=True)


def converged_error(w, iterations: int = 200) -> dict:
    """GPU fp32 against the fp64 oracle after `iterations` with split/join from
    one built state: structure equality, relative energy difference, and the
    mean, sum and maximum of |u_gpu - u_f64| on the finest grid."""
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    o = Oracle("f64").import_state(g.export_state())
    g.fuse(iterations, w.lam, w.tau, w.sigma)
    o.fuse(iterations, w.lam, w.tau, w.sigma)
    eg, eo = g.extract(), o.extract()
    tg, dg = g.energy()
    to, do = o.energy()
    Eg, Eo = tg + w.lam * dg, to + w.lam * do
    D = w.max_depth
    diff = np.abs(to_dense(eg["keys"], eg["levels"], eg["u"].astype(np.float64), D)
                  - to_dense(eo["keys"], eo["levels"], eo["u"], D))
    g.close()
    return dict(same_structure=bool(np.array_equal(eg["keys"], eo["keys"])
                                    and np.array_equal(eg["levels"], eo["levels"])),
                leaves=int(eg["keys"].size), energy_gpu=Eg, energy_f64=Eo, rel_energy=abs(Eg - Eo) / abs(Eo),
                u_l1_mean=float(diff.mean()), u_l1_sum=float(diff.sum()), u_linf=float(diff.max()))


def test_converged_error_against_fp64_oracle():
    r = converged_error(synth.workload(1))
    print(f"fp32 GPU vs fp64 oracle after 200 iterations: {r}", flush=True)
    assert r["same_structure"]
    assert r["rel_energy"] < 1e-6
    assert r["u_linf"] < 1e-5
    assert r["u_l1_mean"] < 1e-6
