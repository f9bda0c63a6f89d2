"""Pins of the oracle's gradient-descent solver (the paper's own method: the
steady state of Eq. 6 on the smoothed energy of Eq. 4-5, lambda on TV).

Each pin ties the step to something other than the step itself: the energy's
numerical derivative, the descent property, and the data-only limit.
"""
from __future__ import annotations

import numpy as np

from oracle import Oracle
from paper_1608_07411_amd import synth
from tests.helpers import base_params, blob_get, blob_set, blob_set_leaves, blob_volumes, parse_views


def _fixed_state(seed=0):
    """Unbalanced octree (depth 5, a thin band around a blob, some voxels
    unobserved) with random u, on a fixed structure."""
    f, w = blob_volumes(3, 5, seed, p_unobs=0.1)
    o = Oracle("f64").build_volumes(f, w, base_params(5, restructure_every=0))
    blob = blob_set(o.export_state(), restructure_every=0)
    _, leaves = parse_views(blob)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=len(leaves)).astype(np.float32)
    return blob_set_leaves(blob, u=u, ubar=u), leaves


def _energy(blob, lam, eps):
    tv, data = Oracle("f64").import_state(blob).energy_eps(eps)
    return data + lam * tv


def test_gd_step_is_the_negative_energy_gradient():
    lam, xi, eps = 0.7, 1e-3, 0.3
    blob, leaves = _fixed_state(0)
    o = Oracle("f64").import_state(blob)
    u0 = o.extract()["u"]
    o.fuse_gd(1, lam, xi, eps)
    direction = (o.extract()["u"] - u0) / xi  # = lambda div q - d'(u)
    rng = np.random.default_rng(1)
    sample = rng.choice(len(u0), size=25, replace=False)
    hstep = 1e-3
    Dmax = blob_get(blob, "max_depth")
    for n in sample:
        up, um = u0.copy(), u0.copy()
        up[n] += hstep
        um[n] -= hstep
        dE = (_energy(blob_set_leaves(blob, u=up), lam, eps) - _energy(blob_set_leaves(blob, u=um), lam, eps)) / (
            2 * hstep)
        vol = float(8 ** (Dmax - int(leaves["level"][n])))
        # u is stored in fp32 in the blob: the perturbation is exact only to fp32, so
        # compare against the slope over the perturbation actually applied
        du = float(np.float32(u0[n] + hstep)) - float(np.float32(u0[n] - hstep))
        dE = dE * (2 * hstep) / du
        assert abs(direction[n] + dE / vol) <= 1e-4 * (1 + abs(direction[n])), (n, direction[n], -dE / vol)


def test_gd_energy_decreases_on_a_fixed_structure():
    lam, xi, eps = 0.5, 0.01, 0.3
    blob, _ = _fixed_state(2)
    o = Oracle("f64").import_state(blob)
    E = []
    for _ in range(40):
        tv, data = o.energy_eps(eps)
        E.append(data + lam * tv)
        o.fuse_gd(1, lam, xi, eps)
    E = np.array(E)
    assert np.all(np.diff(E) < 0), np.diff(E).max()
    assert E[-1] < 0.9 * E[0]


def test_gd_without_regulariser_reaches_each_leafs_single_observation():
    w = synth.sphere_workload(max_depth=4, n_views=1, W=40, H=30, f=37.5, restructure_every=0)
    o = Oracle("f64").build(w.depth, w.cams, w.params)
    obs = o.leaf_obs()
    o.fuse_gd(400, 0.0, 0.01, 0.02)
    u = o.extract()["u"]
    M = obs["M"]
    one = M == 1
    assert one.sum() > 50
    F = obs["F"][obs["off"][:-1][one]]
    assert np.max(np.abs(u[one] - F)) < 1e-4
    # unobserved leaves feel no force without the regulariser
    assert np.all(u[M == 0] == 0.0)


def test_gd_invalid_arguments():
    w = synth.sphere_workload(max_depth=3, n_views=2, W=40, H=30, f=37.5)
    o = Oracle("f64").build(w.depth, w.cams, w.params)
    import pytest
    for bad in ((-1, 0.5, 0.1, 0.1), (1, -0.5, 0.1, 0.1), (1, 0.5, 0.0, 0.1), (1, 0.5, 0.1, 0.0),
                (1, float("nan"), 0.1, 0.1)):
        with pytest.raises(Exception):
            o.fuse_gd(*bad)
