"""Training and evaluation driver of the learned warm start (argument
marshalling around the C ABI; the features, network, training steps and the
solver all run in the library's kernels; torch only holds device buffers).

Training data: plain primal-dual solutions on a frozen structure of the
training spheres (features of each leaf of the initial octree; targets: the
change of the leaf's u and its p after `iterations` iterations).
Evaluation: seconds (and iterations) until the energy E = TV + lambda data
reaches E_ref (1 + 1e-4), E_ref being the plain solver's energy after
`ref_iterations`, from the plain start and from the warm start.
"""
from __future__ import annotations

import time

import numpy as np

from . import otf, synth


def init_params(seed: int, n_params: int) -> np.ndarray:
    """He-normal weights and zero biases for the 32-128-128-128-4 network,
    laid out per layer as W (in x out, row-major) then b."""
    sizes = (32, 128, 128, 128, 4)
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal(a * b) * np.sqrt(2.0 / a)).astype(np.float32))
        parts.append(np.zeros(b, np.float32))
    theta = np.concatenate(parts)
    assert theta.size == n_params
    return theta


def training_set(n_scenes: int, iterations: int, first: int = 0, log=print):
    import torch

    Xs, Ts = [], []
    for j in range(first, first + n_scenes):
        w = synth.warm_training_workload(j)
        c = otf.Context(0).build_octree(torch.from_numpy(w.depth).cuda(), w.cams, w.params)
        X = c.features().cpu().numpy()
        c.fuse(iterations, w.lam, w.tau, w.sigma)
        T = c.targets().cpu().numpy()
        T[:, 0] -= X[:, 22]  # the change of u from its start (feature 22)
        Xs.append(X)
        Ts.append(T)
        c.close()
        if (j - first + 1) % 32 == 0:
            log(f"[warm] {j - first + 1}/{n_scenes} training scenes, {sum(len(x) for x in Xs)} leaves")
    return np.concatenate(Xs), np.concatenate(Ts)


def train(net, X: np.ndarray, T: np.ndarray, epochs: int, batch: int, lr: float, seed: int = 0, log=print):
    """Adam on minibatches of a seeded permutation of the rows (one upload)."""
    import torch

    perm = np.random.default_rng(seed).permutation(len(X))
    Xd = torch.from_numpy(np.ascontiguousarray(X[perm])).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T[perm])).cuda()
    n = len(X)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        tot, cnt = 0.0, 0
        for a in range(0, n - batch + 1, batch):
            tot += net.train_step(Xd[a:a + batch], Td[a:a + batch], lr)
            cnt += 1
        losses.append(tot / max(cnt, 1))
        log(f"[warm] epoch {ep + 1}/{epochs}: mean loss {losses[-1]:.5f}")
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def energy(c, lam: float) -> float:
    tv, data = c.energy()
    return tv + lam * data


def iterations_to_tolerance(c, w, e_target: float, max_iter: int, warm_net=None, alphas=(1.0, 0.5, 0.25)):
    """Iterations until E <= e_target, the energy checked after every
    iteration (not timed), from the plain start or the guarded warm start (the
    network's prediction kept at the step, alphas or none, that lowers the
    energy most). Returns (iterations, reached, alpha)."""
    alpha = None
    if warm_net is not None:
        alpha, _ = c.warm_start_guarded(warm_net, w.lam, alphas)
    for it in range(1, max_iter + 1):
        c.fuse(1, w.lam, w.tau, w.sigma)
        if energy(c, w.lam) <= e_target:
            return it, True, alpha
    return max_iter, False, alpha


def timed_solve(depth, w, iterations: int, warm_net=None, alphas=(1.0, 0.5, 0.25)) -> float:
    """Seconds of the solver from a fresh build (not timed): the guarded warm
    start (if a network is given) and `iterations` iterations, no energy
    checks in between."""
    import torch

    c = otf.Context(0).build_octree(depth, w.cams, w.params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if warm_net is not None:
        c.warm_start_guarded(warm_net, w.lam, alphas)
    c.fuse(iterations, w.lam, w.tau, w.sigma)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    c.close()
    return t


def distance_to_solution(net, scenes, iterations: int):
    """RMS distance of u to the plain solution after `iterations` (frozen
    structure) from the plain start and from the warm start, per scene."""
    import torch

    out = []
    for w in scenes:
        depth = torch.from_numpy(w.depth).cuda()
        c = otf.Context(0).build_octree(depth, w.cams, w.params)
        u0 = c.extract()["u"].astype(np.float64)
        c.warm_start(net)
        uw = c.extract()["u"].astype(np.float64)
        ref = otf.Context(0).build_octree(depth, w.cams, w.params)
        ref.fuse(iterations, w.lam, w.tau, w.sigma)
        us = ref.extract()["u"].astype(np.float64)
        out.append({"scene": w.name, "rms_plain_start": float(np.sqrt(np.mean((u0 - us) ** 2))),
                    "rms_warm_start": float(np.sqrt(np.mean((uw - us) ** 2)))})
        c.close()
        ref.close()
    return out


def evaluate(net, scenes, ref_iterations: int, tol: float = 1e-4, log=print):
    """Per scene: E_ref, the plain solver's energy after ref_iterations; then,
    from the plain start and from the guarded warm start, the iterations until
    E <= E_ref (1 + tol) (the energy checked after every iteration) and the
    seconds of a separate run of exactly that many iterations (warm start
    included, no energy checks)."""
    import torch

    out = []
    for w in scenes:
        depth = torch.from_numpy(w.depth).cuda()
        ref = otf.Context(0).build_octree(depth, w.cams, w.params)
        e0 = energy(ref, w.lam)
        ref.fuse(ref_iterations, w.lam, w.tau, w.sigma)
        e_ref = energy(ref, w.lam)
        leaves = ref.num_leaves()
        ref.close()
        target = e_ref * (1.0 + tol)
        res = {"scene": w.name, "leaves_at_end": leaves, "E_start": e0, "E_ref": e_ref,
               "ref_iterations": ref_iterations}
        for name, nn in (("plain", None), ("warm", net)):
            c = otf.Context(0).build_octree(depth, w.cams, w.params)
            it, ok, alpha = iterations_to_tolerance(c, w, target, 3 * ref_iterations, warm_net=nn)
            c.close()
            res[name] = {"iterations": it, "reached": ok, "seconds": timed_solve(depth, w, it, warm_net=nn)}
            if nn is not None:
                res[name]["alpha"] = alpha
                c2 = otf.Context(0).build_octree(depth, w.cams, w.params)
                res[name]["E_after_warm_start"] = (c2.warm_start_guarded(nn, w.lam)[1])
                c2.close()
        res["speedup"] = res["plain"]["seconds"] / res["warm"]["seconds"]
        log(f"[warm] {w.name}: {res}")
        out.append(res)
    return out
