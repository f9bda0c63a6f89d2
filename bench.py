#!/usr/bin/env python3
"""Throughput of octree TV-L1 range-data fusion on one MI355X.

Metric: leaf-updates per second (sum over iterations of the leaf count, divided
by wall time) on the depth-9 (512^3) thin-structure workload: 64 synthetic
640x480 range maps of slabs, thin cylinders and open shells, 0.5% range noise,
truncation 3 finest voxels, lambda 0.5, tau = sigma = 1/sqrt(12), split and
join after every iteration. One step = one primal-dual iteration (dual sweep,
primal sweep, split/join restructuring) over the whole octree. Inputs are
resident in HBM before the timed region; the octree build is timed
separately. After the warmup the state is exported; --replays (5) timed runs
of --steps iterations each start from it, and the median is reported.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_SOURCES = ("paper_1608_07411_amd/csrc/sweep.hip",)  # the sweep kernels' source
MESH_SOURCES = ("paper_1608_07411_amd/csrc/mesh.hip",)  # the evaluation kernels' source


def traffic_ratio(kernel: str, workload: str, sources=SWEEP_SOURCES):
    """Hardware-to-algorithmic byte ratio of a kernel from its committed profile.

    The profile records FETCH_SIZE/WRITE_SIZE (scaled by a plain copy's
    reading) over algorithmic bytes for the same dispatches, and a hash of the
    kernel's sources; a hash that no longer matches means the kernel has
    changed since the counters were taken, and no ratio is returned.
    """
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path).read().splitlines():
        if " " in line:
            k, v = line.split(" ", 1)
            rec[k] = v.strip()
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in sources)
    if rec.get("source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    try:
        return float(rec["traffic_over_algorithmic"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--replays", type=int, default=5, help="timed replays of --steps iterations from one state")
    ap.add_argument("--workload", default="thin", choices=["thin", "blocks", "sphere", "batch48"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--solver", default="pd", choices=["pd", "gd"],
                    help="pd: primal-dual on the exact energy; gd: the paper's gradient descent (lambda on TV, "
                         "step 0.1 halved every 20 iterations, eps 0.3)")
    ap.add_argument("--cpu-seconds", type=float, default=25.0, help="oracle CPU-baseline budget (fp32 + fp64)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--eval", action="store_true",
                    help="paper-style evaluation on the sphere workload: Eq. 7 quantisation error against a fully "
                         "refined solve for three split/join threshold pairs, and mesh-to-sphere distances")
    ap.add_argument("--convergence", action="store_true",
                    help="per-iteration log (leaf count, splits, joins) and the energy every --log-every iterations "
                         "on the chosen workload (the leaf-count curve the paper plots over the iterations)")
    ap.add_argument("--log-every", type=int, default=10)
    ap.add_argument("--eval-gammas", default="0.01,0.1,1.0",
                    help="--eval: the gamma values (normaliser of Eq. 5) to evaluate")
    ap.add_argument("--warm", action="store_true",
                    help="learned warm start: train the per-leaf network on sphere scenes, then seconds to the plain "
                         "solver's final energy (1e-4 relative) from the plain and the warm start on held-out scenes")
    ap.add_argument("--warm-scenes", type=int, default=2000, help="--warm: training scenes")
    ap.add_argument("--warm-seeds", type=int, default=10, help="--warm: held-out multi-object scenes (seeds from 10000)")
    ap.add_argument("--mesh", action="store_true",
                    help="meshing and Eq. 7 at the finest grid of the chosen workload after --warmup + --steps "
                         "iterations: finest-grid field, quantisation error, marching cubes, --replays times")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer on the GPU 5 times (reference for hardware byte counters)")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch

    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 5}), flush=True)


GD_LAMBDA, GD_STEP0, GD_EPS, GD_HALVE = 0.5, 0.1, 0.3, 20


def gd_step(t: int) -> float:
    """The paper's schedule: step 0.1 halved every 20 iterations (iteration t from 0)."""
    return GD_STEP0 * 0.5 ** (t // GD_HALVE)


class Stepper:
    """Runs iterations of the chosen solver on a context (or the oracle),
    keeping the gradient-descent schedule across calls."""

    def __init__(self, solver: str, w):
        self.solver, self.w, self.t = solver, w, 0

    def run(self, ctx, n: int):
        if self.solver == "pd":
            ctx.fuse(n, self.w.lam, self.w.tau, self.w.sigma)
            self.t += n
            return
        while n > 0:
            k = min(n, GD_HALVE - self.t % GD_HALVE)
            ctx.fuse_gd(k, GD_LAMBDA, gd_step(self.t), GD_EPS)
            self.t += k
            n -= k


def host_cpu() -> dict:
    """The host's CPU model and core counts."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def _oracle_rate(oracle, sub: bytes, w, budget_s: float, precision: str, solver: str, t0_iter: int):
    o = oracle.Oracle(precision).import_state(sub)
    updates, iters = 0, 0
    st = Stepper(solver, w)
    st.t = t0_iter
    t0 = time.perf_counter()
    while True:
        n = o.num_leaves()
        st.run(o, 1)
        updates += n
        iters += 1
        el = time.perf_counter() - t0
        if el >= budget_s or iters >= 1000:
            break
    return updates / el, iters, el


def cpu_baseline(blob: bytes, M, w, budget_s: float, solver: str = "pd", t0_iter: int = 0):
    """The oracle (single-threaded C, pinned to one core) on one aligned cube of
    the GPU state after warmup, cut exactly (every observation mean and weight
    kept) and re-rooted as its own domain: fp32 (the canonical arithmetic the
    GPU follows) and fp64, each for part of the budget."""
    import oracle
    from paper_1608_07411_amd import state

    sub = None
    for level in (3, 4, 2, 1):
        try:
            sub, nleaves, cube = state.crop(blob, level, M=M, min_leaves=2000, max_leaves=400000)
            break
        except ValueError:
            continue
    if sub is None:
        return None
    cpu = host_cpu()
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        r32, it32, el32 = _oracle_rate(oracle, sub, w, 0.6 * budget_s, "f32", solver, t0_iter)
        r64, it64, el64 = _oracle_rate(oracle, sub, w, 0.4 * budget_s, "f64", solver, t0_iter)
    finally:
        os.sched_setaffinity(0, old)
    return {
        "value": r32, "unit": "leaf-updates/s", "cores": 1, "kind": "oracle",
        "fp64_value": r64, "host_cpu": cpu["model"], "nproc": cpu["nproc"], "cpu_count": cpu["cpu_count"],
        "sample": (f"oracle (single-threaded C, pointer octree) pinned to core {core} of {cpu['nproc']} "
                   f"({cpu['model']}), on level-{level} cube #{cube} of the GPU state after warmup ({nleaves} "
                   f"leaves at start, cut exactly: every view stores a node for the cube or a leaf whose count "
                   f"divides by the volume ratio; the cube whose mean observations per leaf is closest to the "
                   f"whole octree's {float(np.mean(M)):.1f}), re-rooted as its own domain, split/join every "
                   f"iteration; fp32 {it32} iterations in {el32:.1f} s, fp64 {it64} iterations in {el64:.1f} s"),
    }


def fp64_check(iterations: int = 200) -> dict:
    """Converged error of the GPU (fp32) against the fp64 oracle on the sphere
    workload (depth 6, 8 range maps 160x120), both from the GPU's built state,
    `iterations` with split/join: structure equality, relative energy
    difference (Eq. 3 with the normaliser of Eq. 5), and |u_gpu - u_f64| on the
    finest grid (mean, sum over voxels, max)."""
    import oracle
    from paper_1608_07411_amd import otf, synth

    w = synth.workload(1)
    g = otf.Context(0).build_octree(w.depth, w.cams, w.params)
    o = oracle.Oracle("f64").import_state(g.export_state())
    g.fuse(iterations, w.lam, w.tau, w.sigma)
    o.fuse(iterations, w.lam, w.tau, w.sigma)
    G = 1 << w.max_depth
    dg = g.dense_field()
    eo = o.extract()
    do = np.zeros(G ** 3)
    x, y, z = oracle.morton_decode(eo["keys"])
    s = 1 << (w.max_depth - eo["levels"].astype(np.int64))
    dense = do.reshape(G, G, G)
    for i in range(len(s)):
        dense[z[i]:z[i] + s[i], y[i]:y[i] + s[i], x[i]:x[i] + s[i]] = eo["u"][i]
    diff = np.abs(np.asarray(dg, np.float64).reshape(-1) - do)
    tg, dag = g.energy()
    to, dao = o.energy()
    Eg, Eo = tg + w.lam * dag, to + w.lam * dao
    eg = g.extract()
    g.close()
    return {"workload": "sphere: depth 6, 8 range maps 160x120, split/join every iteration",
            "iterations": iterations, "leaves": int(eg["keys"].size),
            "same_structure": bool(np.array_equal(eg["keys"], eo["keys"])
                                   and np.array_equal(eg["levels"], eo["levels"])),
            "rel_energy": abs(Eg - Eo) / abs(Eo), "u_l1_mean": float(diff.mean()), "u_l1_sum": float(diff.sum()),
            "u_linf": float(diff.max())}


def stream_ceiling(gib: float = 2.0) -> dict:
    """Plain copy and read rates of this GPU in the same run: a 2 GiB fp32
    buffer copied and summed 5 times each (torch kernels)."""
    import torch

    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    x.sum()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    t_copy = (time.perf_counter() - t0) / 5
    t0 = time.perf_counter()
    for _ in range(5):
        x.sum()
    torch.cuda.synchronize()
    t_read = (time.perf_counter() - t0) / 5
    del x, y
    torch.cuda.empty_cache()
    return {"copy_GBs": 2 * 4 * n / t_copy / 1e9, "read_GBs": 4 * n / t_read / 1e9, "buffer_GiB": gib,
            "note": "torch copy_ (read + write bytes) and sum (read bytes) over a buffer far larger than the caches"}


# --------------------------------------------------------------------------
def run_batch(args):
    """48 sphere objects of depth 6-9 and 8-64 views in one batch (fixed
    structure: no split/join, so the iteration loop is replayed from a HIP
    graph after the autotuner's iterations)."""
    import torch
    from paper_1608_07411_amd import otf, synth

    t0 = time.perf_counter()
    ws = synth.batch_workloads()
    log(f"[bench] {len(ws)} objects generated in {time.perf_counter() - t0:.1f} s")
    depths = [torch.from_numpy(w.depth).cuda() for w in ws]
    torch.cuda.synchronize()
    ctxs = []
    t0 = time.perf_counter()
    for w, d in zip(ws, depths):
        c = otf.Context(0)
        c.build_octree(d, w.cams, w.params)
        ctxs.append(c)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    batch = otf.Batch(0)
    for c in ctxs:
        batch.add(c)
    L = [c.num_leaves() for c in ctxs]
    w0 = ws[0]
    log(f"[bench] built {len(ctxs)} octrees in {build_s:.2f} s, {sum(L)} leaves (min {min(L)}, max {max(L)})")
    batch.fuse(max(args.warmup, 9), w0.lam, w0.tau, w0.sigma)  # includes the autotuner's 9 iterations
    torch.cuda.synchronize()
    cfg = batch.config()
    b0 = [sum(c.profile_read()["bytes"][k] for c in ctxs) for k in ("dual", "primal")]
    t0 = time.perf_counter()
    batch.fuse(args.steps, w0.lam, w0.tau, w0.sigma)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cfg_run = batch.config()
    b1 = [sum(c.profile_read()["bytes"][k] for c in ctxs) for k in ("dual", "primal")]
    alg = (b1[0] - b0[0] + b1[1] - b0[1]) / args.steps
    updates = sum(L) * args.steps
    value = updates / elapsed
    per_it = elapsed / args.steps
    result = {
        "metric": "leaf-updates/sec (48 objects, batched)", "value": value, "unit": "leaf-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": max(args.warmup, 9), "ms_per_step": 1e3 * per_it,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": ("batch48: 48 spheres r=0.3, max depth uniform in {6..9}, 8-64 views 160x120 on a "
                         "circle, seeds 1000-1047, lambda 0.5, tau=sigma=1/sqrt(12), fixed structure"),
            "leaves": sum(L), "launch": cfg, "graph_iterations_timed": cfg_run["graph_iterations"],
        },
        "roofline": {
            "bound": "hbm", "kernel": "batched dual + primal sweeps (whole iteration)", "achieved": alg / per_it / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / per_it / 1e9 / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": alg, "avg_launch_ms": 1e3 * per_it,
        },
        "build_s": build_s,
    }
    if not args.no_cpu:
        import oracle

        k = int(np.argmin(L))
        o = oracle.Oracle("f32").import_state(ctxs[k].export_state())
        n, it, t0 = o.num_leaves(), 0, time.perf_counter()
        while True:
            o.fuse(1, w0.lam, w0.tau, w0.sigma)
            it += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or it >= 1000:
                break
        result["cpu_baseline"] = {
            "value": n * it / el, "unit": "leaf-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle fp32 on batch object {k} ({n} leaves, the smallest), {it} iterations in {el:.1f} s"}
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


def run_eval(args):
    """Sec. 4-style evaluation on the sphere workload (depth 6, 8 views): the
    quantisation error of Eq. 7 between the adaptive octree and a fully refined
    solve over the iterations, for three (split, join) threshold pairs, and the
    distance of the marching-cubes vertices to the true sphere. Two fully
    refined references separate the two sources of the error: one refined
    everywhere down to the data (spread_tau < 0: the view octrees hold every
    finest voxel), and one whose structure is refined but whose data are the
    adaptive view octrees' (split_tau = join_tau = 2: every leaf splits down to
    the finest level in the first iteration and nothing joins). Each for
    gamma in --eval-gammas."""
    import torch
    from paper_1608_07411_amd import otf, synth

    iters = args.steps
    checkpoints = sorted({1, max(1, iters // 4), max(1, iters // 2), iters})
    gammas = [float(g) for g in args.eval_gammas.split(",")]
    out_by_gamma = []
    for gamma in gammas:
        # eta = 3 delta: with the workload's 10 delta (0.47 of the unit domain at
        # depth 6) the solid-behind-the-surface band of Eq. 1's eta rule wraps the
        # whole sphere and moves the zero level off it
        w = synth.sphere_workload(seed=args.seed)
        w.params = dict(w.params, eta=3.0 * w.params["delta"], gamma=gamma)
        depth = torch.from_numpy(w.depth).cuda()
        D = w.max_depth
        h = 2.0 ** -D

        def reference(params):
            ctx = otf.Context(0).build_octree(depth, w.cams, params)
            fields, done = {}, 0
            for k in checkpoints:
                ctx.fuse(k - done, w.lam, w.tau, w.sigma)
                done = k
                f = ctx.dense_field(torch.empty((1 << D) ** 3, dtype=torch.float32, device="cuda"))
                fields[k] = f.clone()
            return ctx, fields

        dense_ctx, ref_dense = reference(dict(w.params, spread_tau=-1.0, join_tau=2.0))
        refd_ctx, ref_refined = reference(dict(w.params, split_tau=2.0, join_tau=2.0))
        torch.cuda.synchronize()

        def sphere_error(ctx):
            xyz, _ = ctx.mesh(0.0)
            v = np.unique(xyz.reshape(-1, 3), axis=0).astype(np.float64)
            prim = w.prims[0]
            if len(v) == 0:
                return dict(vertices=0, mean_voxels=None, std_voxels=None, max_voxels=None)
            d = np.abs(np.linalg.norm(v - prim.c, axis=1) - prim.r) / h
            return dict(vertices=int(len(v)), mean_voxels=float(d.mean()), std_voxels=float(d.std()),
                        median_voxels=float(np.median(d)), within_1_voxel=float((d < 1).mean()),
                        max_voxels=float(d.max()))

        runs = []
        for ts, tj in ((0.0, 0.9), (0.5, 0.9), (0.9, 0.99)):
            ctx = otf.Context(0).build_octree(depth, w.cams, dict(w.params, split_tau=ts, join_tau=tj))
            errs, errs_ref, done, t = {}, {}, 0, 0.0
            for k in checkpoints:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.fuse(k - done, w.lam, w.tau, w.sigma)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
                done = k
                errs[str(k)] = ctx.quantisation_error(ref_dense[k])
                errs_ref[str(k)] = ctx.quantisation_error(ref_refined[k])
            runs.append(dict(split_tau=ts, join_tau=tj, eq7_vs_dense_data=errs, eq7_vs_refined_structure=errs_ref,
                             leaves=ctx.num_leaves(), fuse_s=t, sphere=sphere_error(ctx)))
            log(f"[eval] gamma={gamma} tau_s={ts} tau_j={tj}: Eq.7 vs dense data {errs}, vs refined structure "
                f"over the adaptive data {errs_ref}, {ctx.num_leaves()} leaves")
            ctx.close()
        out_by_gamma.append(dict(gamma=gamma, runs=runs, dense_leaves=dense_ctx.num_leaves(),
                                 dense_sphere=sphere_error(dense_ctx),
                                 refined_structure_leaves=refd_ctx.num_leaves(),
                                 refined_structure_sphere=sphere_error(refd_ctx),
                                 refined_vs_dense=refd_ctx.quantisation_error(ref_dense[iters])))
        dense_ctx.close()
        refd_ctx.close()
    first = out_by_gamma[0]["runs"][1]
    result = {
        "metric": "evaluation (sphere workload)", "value": first["eq7_vs_dense_data"][str(iters)],
        "unit": f"Eq. 7 quantisation error at the last iteration (tau_s 0.5, tau_j 0.9, gamma {gammas[0]}) "
                f"against the fully refined solve over fully refined data", "n_gpus": 1,
        "steps": iters, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sphere: depth 6, 8 views 160x120, lambda 0.5, tau=sigma=1/sqrt(12), eta 3 delta, "
                               f"split/join every iteration", "gammas": gammas},
        "by_gamma": out_by_gamma,
    }
    print(json.dumps(result), flush=True)


def run_warm(args):
    """Learned warm start: training on frozen-structure plain solutions of
    --warm-scenes sphere scenes (radius 0.2-0.35, centre jitter 0.05, depth 6,
    8 views), evaluation on the 10 held-out multi-object scenes (seeds
    10000-10009: depth 8, 32 views 640x480, noise and outliers), with the
    structure frozen and with split/join every iteration, and on 2 held-out
    spheres. Iterations to tolerance are counted with the energy checked after
    every iteration; seconds are timed on separate runs of exactly that many
    iterations."""
    from paper_1608_07411_amd import otf, synth, warm

    n_scenes, epochs = args.warm_scenes, 12
    t0 = time.perf_counter()
    X, T = warm.training_set(n_scenes, 300, log=log)
    t_data = time.perf_counter() - t0
    net = otf.Mlp(0)
    net.set_params(warm.init_params(args.seed, net.n_params))
    losses, t_train = warm.train(net, X, T, epochs, 32768, 1e-3, log=log)
    rows = int(len(X))
    del X, T
    seeds = list(range(10000, 10000 + args.warm_seeds))
    res_frozen = warm.evaluate(net, [synth.blocks_workload(seed=s, restructure_every=0) for s in seeds], 1500, log=log)
    res_split = warm.evaluate(net, [synth.blocks_workload(seed=s, restructure_every=1) for s in seeds], 1500, log=log)
    held_sphere = [synth.warm_training_workload(100000 + k) for k in range(2)]
    res_sphere = warm.evaluate(net, held_sphere, 1500, log=log)

    def gmean(rs):
        return float(np.exp(np.mean([np.log(r["speedup"]) for r in rs])))

    result = {
        "metric": "seconds to energy tol, warm vs plain", "value": gmean(res_frozen),
        "unit": "plain seconds / warm seconds, geometric mean over the 10 held-out multi-object scenes (frozen "
                "structure)", "higher_is_better": True,
        "n_gpus": 1, "steps": None, "dtype": "bf16 network, f32 solver", "data": "synthetic",
        "config": {"workload": (f"train: {n_scenes} sphere scenes (depth 6, 8 views), frozen structure, 300 plain "
                                f"iterations as targets; evaluate: multi-object scenes seeds 10000-"
                                f"{10000 + args.warm_seeds - 1} (depth 8, "
                                f"32 views 640x480) frozen and with split/join every iteration, and 2 held-out "
                                f"spheres; tolerance 1e-4 on the energy after 1500 plain iterations, checked every "
                                f"iteration; the warm start guarded by the energy (steps 1, 0.5, 0.25 or none)"),
                   "training_rows": rows, "epochs": epochs,
                   "data_s": t_data, "train_s": t_train, "final_loss": losses[-1]},
        "speedup_split_join": gmean(res_split), "speedup_spheres": gmean(res_sphere),
        "held_out_frozen": res_frozen, "held_out_split_join": res_split, "held_out_spheres": res_sphere,
    }
    print(json.dumps(result), flush=True)


def run_convergence(args):
    """Leaf count, splits and joins after every iteration, and the energy of
    Eq. 3 with the normaliser of Eq. 5 every --log-every iterations, over
    --steps iterations of the chosen workload with split/join every
    iteration."""
    import torch
    from paper_1608_07411_amd import otf, synth

    maker = {"thin": synth.thin_workload, "blocks": synth.blocks_workload, "sphere": synth.sphere_workload}
    w = maker[args.workload](seed=args.seed)
    depth = torch.from_numpy(w.depth).cuda()
    ctx = otf.Context(0).build_octree(depth, w.cams, w.params)
    tv, da = ctx.energy()
    log_rows = [dict(iteration=0, leaves=ctx.num_leaves(), splits=0, joins=0, energy=tv + w.lam * da, tv=tv, data=da)]
    for it in range(1, args.steps + 1):
        ctx.fuse(1, w.lam, w.tau, w.sigma)
        s_, j_ = ctx.last_counts()
        row = dict(iteration=it, leaves=ctx.num_leaves(), splits=s_, joins=j_)
        if it % args.log_every == 0 or it == args.steps:
            tv, da = ctx.energy()
            row.update(energy=tv + w.lam * da, tv=tv, data=da)
            log(f"[convergence] {row}")
        log_rows.append(row)
    result = {"metric": "convergence log", "workload": f"{w.name}: depth {w.max_depth}, {w.depth.shape[0]} views",
              "steps": args.steps, "log_every": args.log_every, "rows": log_rows}
    print(json.dumps(result), flush=True)


def run_mesh(args):
    """Meshing and Eq. 7 at the finest grid (512^3 voxels on the depth-9 thin
    workload): after --warmup iterations the finest-grid field is kept as the
    reference, --steps more iterations run, then --replays repetitions of the
    finest-grid field (into a device tensor), the quantisation error of Eq. 7
    against the reference field, and marching cubes at iso 0 (the count call,
    then the call that copies the triangles to the host). The field and Eq. 7
    are timed with events on the library's stream (torch's current stream);
    marching cubes, whose output is host memory, by the host clock."""
    import torch

    from paper_1608_07411_amd import otf, synth

    maker = {"thin": synth.thin_workload, "blocks": synth.blocks_workload, "sphere": synth.sphere_workload}
    w = maker[args.workload](seed=args.seed)
    D = w.max_depth
    nvox = 1 << (3 * D)
    ctx = otf.Context(0).build_octree(torch.from_numpy(w.depth).cuda(), w.cams, w.params)
    ctx.fuse(args.warmup, w.lam, w.tau, w.sigma)
    ref = ctx.dense_field(torch.empty(nvox, dtype=torch.float32, device="cuda")).clone()
    ctx.fuse(args.steps, w.lam, w.tau, w.sigma)
    L = ctx.num_leaves()
    out = torch.empty(nvox, dtype=torch.float32, device="cuda")
    log(f"[mesh] {w.name} depth {D}: {L} leaves after {args.warmup} + {args.steps} iterations")

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    def event_timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return 1e-3 * e0.elapsed_time(e1), r

    event_timed(lambda: ctx.dense_field(out))  # first call: the library's scratch grows
    ctx.reset_counters(profile=True)  # the library's own events around each evaluation kernel
    rows = []
    for r in range(max(1, args.replays)):
        t_dense, _ = event_timed(lambda: ctx.dense_field(out))
        t_q, q = event_timed(lambda: ctx.quantisation_error(ref))
        t_mesh, (xyz, ed) = timed(lambda: ctx.mesh(0.0))
        rows.append(dict(dense_ms=1e3 * t_dense, eq7_ms=1e3 * t_q, mesh_ms=1e3 * t_mesh, eq7=q, triangles=len(xyz)))
        log(f"[mesh] replay {r + 1}: {rows[-1]}")
    med = {k: float(np.median([row[k] for row in rows])) for k in ("dense_ms", "eq7_ms", "mesh_ms")}
    kern = {k: dict(v, avg_ms=v["ms"] / max(v["launches"], 1)) for k, v in ctx.profile_read_eval().items()}
    ntri = rows[-1]["triangles"]
    # the finest-grid field: written once (4 B per voxel), every leaf's u and
    # key read once
    dense_bytes = 4 * nvox + 8 * L
    dense_kernel_ms = kern["field"]["avg_ms"]
    achieved = dense_bytes / (dense_kernel_ms * 1e-3) / 1e9
    ratio = traffic_ratio("dense_field", f"{w.name}_depth{D}", MESH_SOURCES)
    result = {
        "metric": "finest voxels meshed per second", "value": nvox / (med["mesh_ms"] * 1e-3), "unit": "voxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: marching cubes and Eq. 7 on the {1 << D}^3 finest grid after "
                               f"{args.warmup} + {args.steps} iterations (split/join every iteration)",
                   "leaves": L, "triangles": ntri, "voxels": nvox},
        "median_ms": med, "eq7": rows[-1]["eq7"],
        "roofline": {"bound": "hbm", "kernel": "k_dense (finest-grid field)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if ratio is None else ratio * dense_bytes,
                     "algorithmic_bytes_per_launch": dense_bytes, "avg_launch_ms": dense_kernel_ms,
                     "bytes_definition": "4 per finest voxel written + 8 per leaf (u and key) read",
                     "timing": "HIP events recorded by the library on its stream around each k_dense launch"},
        "kernel_ms": {k: v["avg_ms"] for k, v in kern.items()},
        "kernel_launches": {k: v["launches"] for k, v in kern.items()},
        "mesh_note": ("mesh_ms: the count call and the call that copies the triangles (36 B of vertices and "
                      "24 B of edge ids each) to the host; each call resamples the field"),
        "replays": rows,
    }
    ctx.close()
    print(json.dumps(result), flush=True)


def main():
    args = parse_args()
    if args.mesh:
        run_mesh(args)
        return
    if args.convergence:
        run_convergence(args)
        return
    if args.warm:
        run_warm(args)
        return
    if args.eval:
        run_eval(args)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "batch48" and args.gpus == 1:
        run_batch(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU; multi-GPU sharding is designed but "
                                   "not built", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    from paper_1608_07411_amd import otf, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    maker = {"thin": synth.thin_workload, "blocks": synth.blocks_workload, "sphere": synth.sphere_workload}
    w = maker[args.workload](seed=args.seed)
    log(f"[bench] workload {w.name}: depth {w.max_depth}, {w.depth.shape[0]} views "
        f"{w.depth.shape[2]}x{w.depth.shape[1]}, generated in {time.perf_counter() - t0:.1f} s")
    depth = torch.from_numpy(w.depth).cuda()
    torch.cuda.synchronize()
    ctx = otf.Context(0)
    t0 = time.perf_counter()
    ctx.build_octree(depth, w.cams, w.params)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    L0 = ctx.num_leaves()
    log(f"[bench] build {build_s:.3f} s, {L0} leaves")
    t0 = time.perf_counter()
    stepper = Stepper(args.solver, w)
    for k in range(args.warmup):
        stepper.run(ctx, 1)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} iterations {time.perf_counter() - t0:.2f} s, {ctx.num_leaves()} leaves, "
        f"last split/join {ctx.last_counts()}")
    # every replay starts from this state
    blob0 = ctx.export_state()
    M0 = ctx.obs_counts()

    def timed_replay(r: int):
        """K iterations from the warmed-up state (re-imported for r > 0); kernel
        events are recorded on the library's stream as it runs."""
        if r > 0:
            ctx.import_state(blob0)
        st = Stepper(args.solver, w)
        st.t = args.warmup
        ctx.reset_counters(profile=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chunk = max(1, args.steps // 5)
        done = 0
        while done < args.steps:
            n = min(chunk, args.steps - done)
            st.run(ctx, n)
            done += n
            log(f"[bench] replay {r + 1}/{args.replays}: {done}/{args.steps} iterations, {ctx.num_leaves()} leaves")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = ctx.profile_read()
        return dict(elapsed=elapsed, prof=prof, value=prof["leaf_updates"] / elapsed, L_end=ctx.num_leaves())

    reps = [timed_replay(r) for r in range(args.replays)]
    order = sorted(range(len(reps)), key=lambda r: reps[r]["value"])
    med = reps[order[len(order) // 2]]
    elapsed, prof = med["elapsed"], med["prof"]
    updates = prof["leaf_updates"]
    value = med["value"]
    L1 = med["L_end"]

    def per_launch(kind):
        n = max(prof[kind]["launches"], 1)
        ms = prof[kind]["ms"] / n
        mb = prof["method_bytes"][kind] / n
        ib = prof["bytes"][kind] / n
        return dict(avg_ms=ms, method_bytes=mb, impl_bytes=ib, method_GBs=mb / (ms * 1e-3) / 1e9,
                    impl_GBs=ib / (ms * 1e-3) / 1e9)

    kern = {k: per_launch(k) for k in ("dual", "primal")}
    sweep_s = (kern["dual"]["avg_ms"] + kern["primal"]["avg_ms"]) * 1e-3
    sweep_bytes = kern["dual"]["method_bytes"] + kern["primal"]["method_bytes"]
    ratio = traffic_ratio({"pd": "leaf_sweep", "gd": "gd_sweep"}[args.solver], f"{w.name}_depth{w.max_depth}")
    names = {"pd": "k_dual + k_primal", "gd": "k_dual (flux) + k_gd_update"}
    achieved = sweep_bytes / sweep_s / 1e9
    roofline = {
        "bound": "hbm", "kernel": f"leaf sweep: {names[args.solver]} (one dual and one primal launch)",
        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": None if ratio is None else ratio * sweep_bytes,
        "traffic_note": ("hardware bytes per sweep = profiled (FETCH_SIZE, WRITE_SIZE)-to-algorithmic ratio x "
                         "this run's algorithmic bytes" if ratio is not None
                         else "no counter profile of the current sweep source"),
        "algorithmic_bytes_per_launch": sweep_bytes, "avg_launch_ms": 1e3 * sweep_s,
        "bytes_definition": ("per leaf-update 40 (u, ubar, p read and written) + 4 per face-adjacency entry + 8 "
                             "(observation offset, normaliser) + 4 per observation + 4 per prefix weight of a "
                             "leaf with fractional weights"),
        "kernels": {f"k_{k}" if args.solver == "pd" else {"dual": "k_dual (flux)", "primal": "k_gd_update"}[k]: v
                    for k, v in kern.items()},
    }
    phase_ms = {k: prof[k]["ms"] for k in ("dual", "primal", "restructure")}
    sweep_ms = phase_ms["dual"] + phase_ms["primal"]
    log(f"[bench] median replay: {updates} leaf-updates in {elapsed:.3f} s -> {value:.4g}/s; phases (ms) {phase_ms}")
    log(f"[bench] sweep {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.3f} of peak); dual {kern['dual']}, "
        f"primal {kern['primal']}")

    result = {
        "metric": "leaf-updates/sec (depth-9 octree)", "value": value, "unit": "leaf-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: octree depth {w.max_depth} ({1 << w.max_depth}^3), {w.depth.shape[0]} range "
                         f"maps {w.depth.shape[2]}x{w.depth.shape[1]}, "
                         + (f"primal-dual, lambda {w.lam}, tau=sigma=1/sqrt(12)" if args.solver == "pd" else
                            f"the paper's gradient descent, lambda {GD_LAMBDA} on TV, step {GD_STEP0} halved every "
                            f"{GD_HALVE} iterations, eps {GD_EPS}")
                         + f", split/join every iteration, seed {args.seed}"),
            "solver": args.solver,
            "leaves_after_build": L0, "leaves_at_end": L1, "mean_leaves_per_step": updates / args.steps,
            "inputs_md5": hashlib.md5(w.depth.tobytes()).hexdigest(),
        },
        "roofline": roofline,
        "replays": {"n": args.replays, "statistic": "median", "from": "one exported state after warmup",
                    "values": [r["value"] for r in reps]},
        "sweep_only": {"value": updates / (sweep_ms * 1e-3) if sweep_ms > 0 else None, "unit": "leaf-updates/s",
                       "note": "dual + primal kernel time only (events), restructuring excluded"},
        "phase_ms": phase_ms, "build_s": build_s,
    }
    ctx.close()
    result["stream_ceiling"] = stream_ceiling()
    log(f"[bench] stream ceiling {result['stream_ceiling']}")
    if not args.no_cpu:
        log("[bench] CPU baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(blob0, M0, w, args.cpu_seconds, args.solver, args.warmup)
        if result["cpu_baseline"]:
            log(f"[bench] CPU baseline {result['cpu_baseline']['value']:.4g} leaf-updates/s (fp32), "
                f"{result['cpu_baseline']['fp64_value']:.4g} (fp64)")
        log("[bench] fp64 check (sphere workload, 200 iterations) ...")
        result["fp64_check"] = fp64_check()
        log(f"[bench] fp64 check {result['fp64_check']}")
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
