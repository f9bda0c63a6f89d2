"""Pins of the oracle's restructuring and of its solver path with fractional
weights, each against a brute force that shares none of its code:

* a join's new leaf carries the block's volume integral of u, ubar and every
  p component (the hierarchical mean over leaves of unequal size);
* a split child inherits u', u_old and p of its parent, its value is the exact
  minimiser of the 1-D prox objective over observations fetched by brute
  force for the child's own box, and its ubar extrapolates from the parent's
  u_old;
* the per-leaf weight total and normaliser equal the brute-force volume
  averages of the view octrees' piecewise-constant weights;
* one primal step on a state with fractional weights gives every leaf the
  exact prox minimiser at its u' (brute-force observations), and u_old is the
  value before the step.

CPU only.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle, morton_decode
from tests.helpers import TAU32, base_params, leaf_boxes, parse_views, plane_volumes
from tests.test_oracle_pins import _brute_min

LAM = 0.5
GAMMA = float(np.float32(1e-2))  # the parameter block holds gamma in fp32


def _view_fields(blob, D, f, w):
    """Per view, the piecewise-constant weight w* and weighted value w*f* of
    its octree's leaves on the finest grid [z, y, x]: the leaves' structure
    from the state, their counts and sums in double from the input volumes."""
    views, _ = parse_views(blob)
    G = 1 << D
    out = []
    for v, nodes in enumerate(views):
        W = np.zeros((G, G, G))
        WF = np.zeros((G, G, G))
        fv = f[v].astype(np.float64) * w[v]
        for n in nodes[nodes["leaf"] == 1]:
            x, y, z = (int(a[0]) for a in morton_decode(np.array([n["key"]])))
            s = 1 << (D - int(n["level"]))
            sl = np.s_[z:z + s, y:y + s, x:x + s]
            W[sl] = float(w[v][sl].sum()) / s ** 3
            WF[sl] = float(fv[sl].sum()) / s ** 3
        out.append((W, WF))
    return out


def _bf_obs(fields, x, y, z, s):
    """(F, W) of every view with a positive volume-averaged weight over the box."""
    sl = np.s_[z:z + s, y:y + s, x:x + s]
    F, W = [], []
    for Wv, WFv in fields:
        w = Wv[sl].mean()
        if w > 0:
            W.append(w)
            F.append(WFv[sl].mean() / w)
    return np.array(F), np.array(W)


def _bf_prox(fields, x, y, z, s, uprime):
    F, W = _bf_obs(fields, x, y, z, s)
    t = float(TAU32) * LAM / (W.sum() + GAMMA)
    return _brute_min(uprime, F, W, t)[0] if len(F) else uprime


def _step_and_restructure(D=4, seed=7):
    """A state (plane volumes, 30% unobserved voxels) after one primal-dual
    iteration without restructuring, and the same after its split/join."""
    f, w = plane_volumes(3, D, seed, p_unobs=0.3)
    a = Oracle("f64").build_volumes(f, w, base_params(D, restructure_every=0))
    fields = _view_fields(a.export_state(), D, f, w)
    before = a.extract()
    a.fuse(1, LAM, TAU32, TAU32)
    pre, pre_aux = a.extract(), a.extract_aux()
    a.restructure_now(LAM, TAU32)
    post, post_aux = a.extract(), a.extract_aux()
    return fields, before, pre, pre_aux, post, post_aux


def _containing(pre, D, X, Y, Z, S):
    x, y, z, s = leaf_boxes(pre["keys"], pre["levels"], D)
    return np.nonzero((x >= X) & (x < X + S) & (y >= Y) & (y < Y + S) & (z >= Z) & (z < Z + S))[0]


def _parent_of(pre, D, X, Y, Z):
    x, y, z, s = leaf_boxes(pre["keys"], pre["levels"], D)
    hit = np.nonzero((X >= x) & (X < x + s) & (Y >= y) & (Y < y + s) & (Z >= z) & (Z < z + s))[0]
    assert len(hit) == 1
    return int(hit[0])


def test_join_keeps_block_integrals():
    D = 4
    _, _, pre, _, post, _ = _step_and_restructure(D)
    px, py, pz, ps = leaf_boxes(post["keys"], post["levels"], D)
    _, _, _, s_pre = leaf_boxes(pre["keys"], pre["levels"], D)
    vol_pre = s_pre.astype(np.float64) ** 3
    n_join = n_mixed = 0
    for j in range(len(px)):
        inside = _containing(pre, D, px[j], py[j], pz[j], ps[j])
        if len(inside) <= 1:
            continue
        n_join += 1
        n_mixed += len(set(pre["levels"][inside].tolist())) > 1
        assert vol_pre[inside].sum() == float(ps[j]) ** 3  # the block is tiled
        vol = float(ps[j]) ** 3
        for name, col in (("u", None), ("ubar", None), ("p", 0), ("p", 1), ("p", 2)):
            v_pre = pre[name][inside] if col is None else pre[name][inside, col]
            v_post = post[name][j] if col is None else post[name][j, col]
            integral = float(np.sum(vol_pre[inside] * v_pre))
            assert abs(vol * v_post - integral) <= 1e-12 * (abs(integral) + vol), (name, col)
    # joins happened, some over leaves of unequal size (where a plain mean over
    # the leaves would differ from the hierarchical one)
    assert n_join >= 10 and n_mixed >= 2


def test_split_children_inherit_and_run_their_own_prox():
    D = 4
    fields, before, pre, pre_aux, post, post_aux = _step_and_restructure(D)
    pk = set(zip(pre["keys"].tolist(), pre["levels"].tolist()))
    px, py, pz, ps = leaf_boxes(post["keys"], post["levels"], D)
    n_kids = n_deep = 0
    for j in range(len(px)):
        if (int(post["keys"][j]), int(post["levels"][j])) in pk:
            continue
        inside = _containing(pre, D, px[j], py[j], pz[j], ps[j])
        if len(inside) > 1:
            continue  # a join
        par = _parent_of(pre, D, px[j], py[j], pz[j])
        assert pre_aux["split"][par] and post["levels"][j] > pre["levels"][par]
        n_kids += 1
        n_deep += int(post["levels"][j]) > int(pre["levels"][par]) + 1
        # inherited: u', u_old, p (copies)
        assert post_aux["uprime"][j] == pre_aux["uprime"][par]
        assert post_aux["uold"][j] == pre_aux["uold"][par]
        assert np.array_equal(post["p"][j], pre["p"][par])
        # u_old is the parent's value before the step
        assert pre_aux["uold"][par] == before["u"][par]
        # own prox: exact minimiser with brute-force observations of the child's box
        u_bf = _bf_prox(fields, px[j], py[j], pz[j], ps[j], pre_aux["uprime"][par])
        assert abs(post["u"][j] - u_bf) < 1e-9
        assert abs(post["ubar"][j] - (2.0 * post["u"][j] - before["u"][par])) < 1e-12
        # the cascade stops where the child is no longer flagged
        assert abs(post["u"][j]) >= 0.5 or post["levels"][j] == D
    assert n_kids >= 100 and n_deep >= 8


@pytest.mark.parametrize("iters", [0, 3])
def test_weight_total_and_normaliser_bruteforce(iters):
    D = 4
    f, w = plane_volumes(3, D, 7, p_unobs=0.3)
    o = Oracle("f64").build_volumes(f, w, base_params(D))
    init = o.extract()
    o.fuse(iters, LAM, TAU32, TAU32)
    fields = _view_fields(o.export_state(), D, f, w)
    ex, ob = o.extract(), o.leaf_obs()
    x, y, z, s = leaf_boxes(ex["keys"], ex["levels"], D)
    n_frac = 0
    for i in range(len(x)):
        F, W = _bf_obs(fields, x[i], y[i], z[i], s[i])
        assert abs(ob["wtot"][i] - W.sum()) < 1e-12
        assert abs(ob["inv"][i] - 1.0 / (W.sum() + GAMMA)) < 1e-9
        n_frac += bool(np.any((W > 0) & (W < 1)))
        if iters == 0:
            # start value: the normalised weighted mean of the observations
            assert abs(init["u"][i] - np.sum(W * F) / (W.sum() + GAMMA)) < 1e-9
    assert n_frac > len(x) // 10


def test_primal_step_with_fractional_weights_is_exact_prox():
    D = 4
    fields, before, pre, pre_aux, _, _ = _step_and_restructure(D)
    x, y, z, s = leaf_boxes(pre["keys"], pre["levels"], D)
    n_frac = 0
    for i in range(len(x)):
        F, W = _bf_obs(fields, x[i], y[i], z[i], s[i])
        n_frac += bool(np.any((W > 0) & (W < 1)))
        assert pre_aux["uold"][i] == before["u"][i]
        u_bf = _bf_prox(fields, x[i], y[i], z[i], s[i], pre_aux["uprime"][i])
        assert abs(pre["u"][i] - u_bf) < 1e-9
        assert abs(pre["ubar"][i] - (2.0 * pre["u"][i] - before["u"][i])) < 1e-12
    assert n_frac > len(x) // 10


def test_initial_structure_is_union_of_view_structures():
    """The fused octree starts as the union of the view octrees: its inner
    nodes (the proper ancestors of its leaves) are exactly the nodes that some
    view splits."""
    D = 5
    f, w = plane_volumes(3, D, 11, p_unobs=0.2)
    o = Oracle("f64").build_volumes(f, w, base_params(D))
    views, leaves = parse_views(o.export_state())
    split = set()
    for nodes in views:
        for n in nodes[nodes["leaf"] == 0]:
            split.add((int(n["level"]), int(n["key"])))
    inner = set()
    for k, lv in zip(leaves["key"].tolist(), leaves["level"].tolist()):
        for L in range(lv):
            inner.add((L, k & ~((1 << (3 * (D - L))) - 1)))
    assert len(split) > 50
    assert inner == split
