"""The full-size workload in the configuration bench.py times (depth-9 thin
structures, 64 range maps 640x480, ~1.3e7 leaves), checked where the oracle
cannot run whole: on sampled leaves the oracle computes one by one, and by
properties that hold at any size.

* Prox: two contexts built from the same inputs take the same frozen-structure
  warmup; then one iteration with lambda and one with lambda = 0. The dual step
  does not depend on lambda, and with lambda = 0 the prox returns u' itself, so
  the second context yields each leaf's u'. For 4096 sampled leaves the
  oracle's prox of their observations (fetched from the device) at that u'
  must equal the first context's u bit for bit.
* A cube of the full-size state: after 5 iterations with split and join a
  level-3 cube (64^3 finest voxels) is cut out of the exported state with
  every observation mean and weight kept exactly, and re-rooted as its own
  domain. Its leaves' observations fetched by the oracle from the cut view
  octrees equal those the GPU fetched at full size; then one iteration with
  split and join on the GPU and in the fp32 oracle from that state (the
  dual step, divergence, prox, split/join decisions and the fetch of new
  leaves) and 5 more, bit for bit.
* Evaluation at full size (the 512^3 finest grid): the field and the
  marching-cubes vertex set on sampled boxes around mesh vertices against the
  oracle's box forms, bit for bit; Eq. 7 is 0 against the own field and,
  against the field of the same leaves with perturbed values u', equals the
  sum of |u - u'| (the mean of a constant over a leaf is exact).
* Structure and dual feasibility after iterations with split and join: the
  leaves tile the domain in Morton order, every p has norm at most 1 (up to
  one rounding), and every leaf has |u| >= tau_s or lies at the maximum depth
  (a flagged leaf splits until that holds, a collapse takes means of values
  beyond tau_j >= tau_s of one sign).
"""
import numpy as np
import pytest

import oracle
from oracle import mesh as om
from paper_1608_07411_amd import state, synth
from tests.helpers import blob_set_leaves

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


@pytest.fixture(scope="module")
def work():
    print("full-size workload: thin, depth 9, 64 views 640x480", flush=True)
    return synth.thin_workload(seed=0)


def _tiles_domain(keys, levels, D):
    size = np.left_shift(np.ones(keys.size, np.int64), 3 * (D - levels.astype(np.int64)))
    k = keys.astype(np.int64)
    return bool(k[0] == 0 and np.all(k[1:] == k[:-1] + size[:-1]) and k[-1] + size[-1] == 1 << (3 * D)
                and np.all(k % size == 0))


def test_full_size_prox_on_sampled_leaves(work):
    w = work
    prm = dict(w.params, restructure_every=0)
    dev = torch.from_numpy(w.depth).cuda()
    a = otf.Context(0).build_octree(dev, w.cams, prm)
    b = otf.Context(0).build_octree(dev, w.cams, prm)
    for c in (a, b):
        c.fuse(3, w.lam, w.tau, w.sigma)
    a.fuse(1, w.lam, w.tau, w.sigma)
    b.fuse(1, 0.0, w.tau, w.sigma)
    ea, eb = a.extract(), b.extract()
    assert np.array_equal(ea["keys"], eb["keys"])
    L = ea["keys"].size
    print(f"leaves {L}", flush=True)
    assert L > 10_000_000
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(L, 4096, replace=False))
    ob = a.extract_obs_at(idx)
    tl = float(np.float32(np.float32(w.tau) * np.float32(w.lam)))
    checked = 0
    for t, i in enumerate(idx):
        up = float(eb["u"][i])
        if up == 0.0:  # a signed zero is not observable through the lambda = 0 run
            continue
        s0, s1 = ob["off"][t], ob["off"][t + 1]
        F = ob["F"][s0:s1].astype(np.float64)
        W = ob["W"][s0:s1].astype(np.float64)
        want = oracle.prox(F, W, w.params["gamma"], up, tl, precision="f32")
        assert np.float32(want) == ea["u"][i], f"leaf {i}: {ea['u'][i]!r} != {want!r}"
        checked += 1
    assert checked > 4000
    a.close()
    b.close()


def test_full_size_structure_after_split_join(work):
    w = work
    D = w.max_depth
    dev = torch.from_numpy(w.depth).cuda()
    c = otf.Context(0).build_octree(dev, w.cams, w.params)
    for k in range(3):
        c.fuse(2, w.lam, w.tau, w.sigma)
        ex = c.extract()
        print(f"after {2 * (k + 1)} iterations: {ex['keys'].size} leaves, last split/join {c.last_counts()}",
              flush=True)
        assert _tiles_domain(ex["keys"], ex["levels"], D)
        pn = np.sqrt(np.sum(ex["p"].astype(np.float64) ** 2, axis=1))
        assert pn.max() <= 1.0 + 1e-6
        ok = (np.abs(ex["u"]) >= np.float32(w.params["split_tau"])) | (ex["levels"] == D)
        assert ok.all(), f"{np.count_nonzero(~ok)} leaves below tau_s above max depth"
    assert sum(c.last_counts()) > 0
    c.close()


def test_full_size_cube_parity(work):
    w = work
    dev = torch.from_numpy(w.depth).cuda()
    c = otf.Context(0).build_octree(dev, w.cams, w.params)
    c.fuse(5, w.lam, w.tau, w.sigma)
    blob = c.export_state()
    M = c.obs_counts()
    sub = None
    for level in (3, 4, 2):
        try:
            sub, n, cube = state.crop(blob, level, M=M, min_leaves=20000, max_leaves=400000)
            break
        except ValueError:
            continue
    assert sub is not None, "no cube can be cut exactly"
    print(f"level-{level} cube #{cube}: {n} leaves", flush=True)
    D = w.max_depth
    keys = state.parse(blob)[2]["key"]
    idx = np.nonzero((keys.astype(np.int64) >> (3 * (D - level))) == cube)[0]
    full = c.extract_obs_at(idx)
    c.close()
    del blob
    o = oracle.Oracle("f32").import_state(sub)
    ob = o.leaf_obs()
    assert np.array_equal(ob["M"], full["M"])
    assert np.array_equal(ob["F"], full["F"].astype(np.float64))
    assert np.array_equal(ob["W"], full["W"].astype(np.float64))
    assert np.array_equal(ob["inv"], full["inv"].astype(np.float64))
    g = otf.Context(0).import_state(sub)
    assert g.export_state() == o.export_state()
    for it in range(6):
        g.fuse(1, w.lam, w.tau, w.sigma)
        o.fuse(1, w.lam, w.tau, w.sigma)
        assert g.last_counts() == o.last_counts(), f"iteration {it + 1}: split/join counts"
        if it in (0, 5):
            assert g.export_state() == o.export_state(), f"state after {it + 1} iterations"
    print(f"cube: 6 iterations identical, {g.num_leaves()} leaves", flush=True)
    g.close()


def test_full_size_evaluation_on_sampled_boxes(work):
    w = work
    D = w.max_depth
    G = 1 << D
    c = otf.Context(0).build_octree(torch.from_numpy(w.depth).cuda(), w.cams, w.params)
    c.fuse(4, w.lam, w.tau, w.sigma)
    lv = c.extract()
    L = lv["keys"].size
    field = c.dense_field(torch.empty(G ** 3, dtype=torch.float32, device="cuda")).view(G, G, G)
    xyz, ed = c.mesh(0.0)
    print(f"full-size evaluation: {L} leaves, {len(xyz)} triangles", flush=True)
    assert len(xyz) > 10000
    ids = ed.reshape(-1)
    pts = xyz.reshape(-1, 3)
    rng = np.random.default_rng(7)
    n = 24
    for k in rng.choice(ids.size, 4, replace=False):
        vox = int(ids[k]) // 3
        v = (vox % G, (vox // G) % G, vox // (G * G))
        origin = tuple(min(max(0, int(a) - n // 2), G - n) for a in v)
        ox, oy, oz = origin
        box = om.dense_box(lv["keys"], lv["levels"], lv["u"], D, origin, (n, n, n))
        assert np.array_equal(field[oz:oz + n, oy:oy + n, ox:ox + n].cpu().numpy(), box)
        bid, bpos = om.crossing_vertices(box, 0.0, D, origin)
        vv, ax = ids // 3, ids % 3
        vx, vy, vz = vv % G, (vv // G) % G, vv // (G * G)
        inside = ((vx >= ox) & (vx + (ax == 0) < ox + n) & (vy >= oy) & (vy + (ax == 1) < oy + n)
                  & (vz >= oz) & (vz + (ax == 2) < oz + n))
        gid, first = np.unique(ids[inside], return_index=True)
        assert len(bid) > 0
        assert np.array_equal(gid, bid)
        assert np.array_equal(pts[inside][first], bpos)
    assert c.quantisation_error(field.view(-1)) == 0.0
    # the same leaves with values moved by multiples of 2^-12 in [-0.5, 0.5]
    d = (rng.integers(-2048, 2049, L) * 2.0 ** -12).astype(np.float32)
    u2 = (lv["u"] + d).astype(np.float32)
    other = otf.Context(0).import_state(blob_set_leaves(c.export_state(), u=u2))
    field2 = other.dense_field(torch.empty(G ** 3, dtype=torch.float32, device="cuda"))
    other.close()
    e = c.quantisation_error(field2)
    e_ref = float(np.sum(np.abs(lv["u"].astype(np.float64) - u2.astype(np.float64))))
    assert abs(e - e_ref) <= 1e-12 * e_ref
    c.close()
