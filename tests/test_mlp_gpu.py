"""The warm-start network on the GPU (MFMA kernels) against the numpy oracle:
forward outputs, loss and gradients (to bf16 accuracy: the two sides round
the same values to bf16 but accumulate in different orders), training that
lowers the loss, features against their definition, and the warm start."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from oracle import mlp as om
from paper_1608_07411_amd import synth
from tests.helpers import TAU32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - the GPU suite runs on the MI355X machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_07411_amd import otf  # noqa: E402


def _data(rows, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, 32)).astype(np.float32)
    T = rng.standard_normal((rows, 4)).astype(np.float32)
    return X, T


def _hidden_outputs(theta, X, layer):
    """The GPU's hidden activations of `layer` (1..3), exactly: the layers
    after it pass their input through (identity weights, zero bias: one exact
    product per sum, and ReLU and bf16 leave a non-negative bf16 value
    unchanged) and the output layer selects 4 units at a time."""
    sizes = om.SIZES
    parts = om.unpack(theta)
    Xd = torch.from_numpy(X).cuda()
    net = otf.Mlp(0)
    H = np.zeros((X.shape[0], sizes[layer]), np.float64)
    for s0 in range(0, sizes[layer], 4):
        vec = []
        for li, (W, b) in enumerate(parts):
            if li < layer:
                vec += [W.ravel(), b]
            elif li < len(parts) - 1:
                vec += [np.eye(sizes[li], dtype=np.float32).ravel(), np.zeros(sizes[li + 1], np.float32)]
            else:
                sel = np.zeros((sizes[li], 4), np.float32)
                sel[np.arange(s0, s0 + 4), np.arange(4)] = 1.0
                vec += [sel.ravel(), np.zeros(4, np.float32)]
        net.set_params(np.concatenate(vec).astype(np.float32))
        H[:, s0:s0 + 4] = net.forward(Xd).cpu().numpy()
    net.close()
    return H


def _device_layers(theta, X):
    """bf16(X), the GPU's three hidden activations and its outputs."""
    net = otf.Mlp(0)
    net.set_params(theta)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    net.close()
    return [om.bf16(X).astype(np.float64)] + [_hidden_outputs(theta, X, l) for l in (1, 2, 3)], Y


def test_forward_matches_oracle_per_element():
    """Layer by layer from the GPU's own inputs to that layer: every hidden
    activation lies in the interval of bf16 values that a sum of the same
    fp32 products in any order can round to (per element), and every output
    within that sum's rounding bound; the two sides differ only where the
    order of the fp32 sum decides a bf16 rounding."""
    theta = om.init_params(5)
    net = otf.Mlp(0)
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    net.close()
    parts = om.unpack(theta)
    for rows in (1, 17, 1000):
        X, _ = _data(rows, rows)
        acts, Y = _device_layers(theta, X)
        flips = 0
        for li in range(3):
            v, lo, hi = om.layer_interval(acts[li], *parts[li], hidden=True)
            dev = acts[li + 1]
            assert np.all((dev >= lo) & (dev <= hi)), (rows, li)
            flips += int(np.count_nonzero(dev != v))
        z, lo, hi = om.layer_interval(acts[3], *parts[3], hidden=False)
        Y = Y.astype(np.float64)
        assert np.all((Y >= lo) & (Y <= hi)), rows
        R, _ = om.forward(theta, X)
        print(f"{rows} rows: {flips} hidden values differ in their bf16 rounding; outputs within "
              f"{np.max(np.abs(Y - z)):.3g} of the oracle given the same inputs (bound {np.max(hi - z):.3g}), "
              f"{np.max(np.abs(Y - R)):.3g} from the oracle's own forward", flush=True)


def test_gradient_matches_oracle_per_element():
    """Every gradient element within its own bound: from the GPU's activations
    and outputs, the oracle forms the device's dZ exactly, and bounds each
    product sum over the rows and each bf16 rounding of the backward pass
    (per element, tight where no rounding is in doubt)."""
    theta = om.init_params(7)
    X, T = _data(6000, 1)  # long enough for the split reduction over rows
    acts, Y = _device_layers(theta, X)
    net = otf.Mlp(0)
    net.set_params(theta)
    loss, g = net.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    net.close()
    want, bound = om.grad_bound(theta, X, T, acts=acts, Y=Y)
    dev = np.abs(g.astype(np.float64) - want)
    assert np.all(dev <= bound), np.argmax(dev - bound)
    rel = np.median(bound / np.maximum(np.abs(want), 1e-12))
    ratio = np.max(np.where(bound > 0, dev / np.where(bound > 0, bound, 1.0), 0.0))
    print(f"gradient: max deviation {dev.max():.3g}, max deviation / bound {ratio:.3g}, "
          f"median bound / |gradient| {rel:.3g}", flush=True)
    assert rel < 1e-2
    # the loss from the GPU's own outputs: fp32 differences, squares summed in double
    d = (Y.astype(np.float32) - T.astype(np.float32)).astype(np.float64)
    assert abs(loss - np.mean(d * d)) <= 1e-12 * loss


def test_training_lowers_the_loss():
    net = otf.Mlp(0)
    net.set_params(om.init_params(11))
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4096, 32)).astype(np.float32)
    # targets from a fixed smooth function of the inputs
    T = np.stack([np.tanh(X[:, :8].sum(1) / 3), np.sin(X[:, 8]), 0.5 * X[:, 9] * X[:, 10], X[:, 11] ** 2 / 4],
                 axis=1).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    first = net.train_step(Xd, Td, 1e-3)
    for _ in range(300):
        last = net.train_step(Xd, Td, 1e-3)
    assert last < 0.2 * first, (first, last)


def _oracle_features(g):
    lv = g.extract()
    o = Oracle("f32").import_state(g.export_state())
    obs = o.leaf_obs()
    counts, idx = o.neighbours()
    L = len(lv["u"])
    X = np.zeros((L, 32), np.float64)
    off = np.concatenate([[0], np.cumsum(counts.sum(1))])
    u = lv["u"].astype(np.float64)
    for i in range(L):
        M, o0 = obs["M"][i], obs["off"][i]
        for k in range(16):
            X[i, k] = obs["F"][o0 + ((2 * k + 1) * M) // 32] if M else 0.0
        at = off[i]
        for f in range(6):
            nb = idx[at:at + counts[i, f]]
            at += counts[i, f]
            X[i, 16 + f] = u[nb].mean() if len(nb) else 0.0
        X[i, 22] = u[i]
        X[i, 23] = obs["wtot"][i] / (obs["wtot"][i] + 1e-2)
        X[i, 24] = M / 64.0
        X[i, 25] = lv["levels"][i] / 5.0
    return X


def test_features_match_their_definition():
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    g.fuse(3, 0.5, TAU32, TAU32)
    X = g.features().cpu().numpy()
    R = _oracle_features(g)
    assert np.max(np.abs(X - R)) < 1e-5


def test_warm_start_writes_the_prediction():
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0, restructure_every=0)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    net = otf.Mlp(0)
    net.set_params(om.init_params(13) * 0.3)
    Y = net.forward(g.features()).cpu().numpy()
    u0 = g.extract()["u"]
    g.warm_start(net)
    lv = g.extract()
    want = np.clip(u0 + Y[:, 0], -1.0, 1.0).astype(np.float32)
    assert np.array_equal(lv["u"], want) and np.array_equal(lv["ubar"], want)
    q = Y[:, 1:].astype(np.float64)
    n = np.sqrt((q ** 2).sum(1))
    assert np.all(np.sqrt((lv["p"].astype(np.float64) ** 2).sum(1)) <= 1.0 + 1e-6)
    inside = n <= 1.0
    assert np.array_equal(lv["p"][inside], Y[inside, 1:])
    g.fuse(5, 0.5, TAU32, TAU32)  # the solver runs from the warm state


def test_trained_warm_start_moves_u_toward_the_solution():
    """What the trained network gains: on held-out spheres of the training
    family, the warm-started u lies closer (RMS) to the plain solver's
    solution than the plain start does."""
    from paper_1608_07411_amd import warm

    X, T = warm.training_set(24, 200, log=lambda *a: None)
    net = otf.Mlp(0)
    net.set_params(om.init_params(0))
    losses, _ = warm.train(net, X, T, 6, 16384, 1e-3, log=lambda *a: None)
    assert losses[-1] < 0.7 * losses[0]
    res = warm.distance_to_solution(net, [synth.warm_training_workload(90000 + k) for k in range(2)], 200)
    for r in res:
        assert r["rms_warm_start"] < 0.9 * r["rms_plain_start"], r


def _energy(g, lam):
    tv, data = g.energy()
    return tv + lam * data


@pytest.mark.parametrize("scale", [0.3, 3.0])
def test_guarded_warm_start_keeps_the_lowest_energy(scale):
    """The guarded warm start against the plain warm start on twin contexts:
    the kept state is the candidate (alpha 1, 0.5 or the current state) of
    lowest energy, bit for bit; a network far off (scale 3) is rejected when
    every candidate raises the energy."""
    lam = 0.5
    w = synth.sphere_workload(max_depth=5, n_views=4, W=80, H=60, f=75.0, restructure_every=0)
    net = otf.Mlp(0)
    net.set_params(om.init_params(13) * scale)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    g.fuse(3, lam, TAU32, TAU32)
    st = g.extract()
    e_plain = _energy(g, lam)
    Y = net.forward(g.features()).cpu().numpy()
    # candidate alpha = 1: the plain warm start on a twin context
    t = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    t.fuse(3, lam, TAU32, TAU32)
    t.warm_start(net)
    e_one = _energy(t, lam)
    one = t.extract()
    a, e = g.warm_start_guarded(net, lam, (1.0, 0.5))
    lv = g.extract()
    assert a in (0.0, 0.5, 1.0)
    assert e <= e_plain and e <= e_one
    assert abs(_energy(g, lam) - e) <= 1e-9 * max(1.0, abs(e))
    if a == 1.0:
        for k in ("u", "ubar", "p"):
            assert np.array_equal(lv[k], one[k]), k
    elif a == 0.0:
        assert e == e_plain and e_one >= e_plain
        for k in ("u", "ubar", "p"):
            assert np.array_equal(lv[k], st[k]), k
    else:
        want = np.clip(np.float32(0.5) * Y[:, 0] + st["u"], -1.0, 1.0)
        assert np.array_equal(lv["u"], want.astype(np.float32)) and e < min(e_plain, e_one)
    g.fuse(5, lam, TAU32, TAU32)  # the solver runs from the kept state


def _small_trained_network():
    from paper_1608_07411_amd import warm

    X, T = warm.training_set(24, 300, log=lambda *a: None)
    net = otf.Mlp(0)
    net.set_params(om.init_params(0))
    warm.train(net, X, T, 6, 16384, 1e-3, log=lambda *a: None)
    return net


def test_warm_start_reaches_the_tolerance_sooner_on_held_out_spheres():
    """Time to the plain solver's energy (1e-4 relative, the energy checked
    every iteration) from the guarded warm start against the plain start, on
    held-out spheres of the training family: fewer iterations."""
    from paper_1608_07411_amd import warm

    net = _small_trained_network()
    scenes = [synth.warm_training_workload(100000 + k) for k in range(2)]
    for r in warm.evaluate(net, scenes, 1500, log=lambda *a: None):
        assert r["plain"]["reached"] and r["warm"]["reached"], r
        assert r["warm"]["iterations"] < r["plain"]["iterations"], r


@pytest.mark.xfail(strict=False, reason="a measured negative result: the network trained on sphere scenes does "
                                        "not shorten the solve of held-out multi-object scenes (0.89x the plain "
                                        "solver's speed over ten such scenes with the full training set)")
def test_warm_start_is_faster_on_a_held_out_multi_object_scene():
    """The same on a held-out multi-object scene (depth 8, 32 views, frozen
    structure): the warm start should take fewer seconds than the plain start
    to the plain solver's energy after 300 iterations."""
    from paper_1608_07411_amd import warm

    net = _small_trained_network()
    r = warm.evaluate(net, [synth.blocks_workload(seed=10000, restructure_every=0)], 300, log=lambda *a: None)[0]
    assert r["plain"]["reached"] and r["warm"]["reached"], r
    assert r["speedup"] > 1.0, r
