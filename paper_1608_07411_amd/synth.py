"""Seeded synthetic range data: scenes, pinhole cameras and ray-cast depth maps.

This module only generates inputs. It holds none of the fusion method's
arithmetic: no TSDF, no octree, no solver. Both the HIP path and the CPU oracle
consume what it produces, so it must stay free of anything either of them
computes.

The paper's own data (rendered sphere views, Carmine 1.09 sequences, the GIS
turbine blade scans; Sec. 4) are not available. The workloads below stand in
for them with analytic primitives rendered into depth maps that hold the radial
range along each pixel-centre ray, which is what the signed distance of Eq. 1
compares against (it uses the Euclidean distance to the projection centre).

Randomness: SplitMix64 (Steele, Lea, Flood 2014) in counter form. A stream is
keyed by (workload, seed, purpose); uniforms are (x >> 11) * 2^-53 and
Gaussians use the cosine branch of Box-Muller.

Geometry is written with explicit element-wise arithmetic in a fixed order (no
BLAS products), so that the same seed gives the same range maps on any host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# SplitMix64
# ----------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _mix_int(z: int) -> int:
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def stream_key(workload: int, seed: int, purpose: int) -> int:
    """Initial SplitMix64 state of the stream for (workload, seed, purpose)."""
    s = _mix_int(0x1608_0741_1000_0000 + workload)
    s = _mix_int(s ^ (seed * 0x9E3779B97F4A7C15))
    return _mix_int(s ^ ((purpose + 1) * 0xD1B54A32D192ED03))


class Stream:
    """Counter-based SplitMix64: output i is mix(state0 + (i + 1) * gamma)."""

    def __init__(self, workload: int, seed: int, purpose: int):
        self.state0 = np.uint64(stream_key(workload, seed, purpose))
        self.counter = 0

    def raw(self, n: int) -> np.ndarray:
        idx = np.arange(self.counter + 1, self.counter + 1 + n, dtype=np.uint64)
        self.counter += n
        with np.errstate(over="ignore"):
            x = self.state0 + idx * _GAMMA
        return _mix(x)

    def uniform(self, n: int = 1, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.raw(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def normal(self, n: int) -> np.ndarray:
        u1 = 1.0 - self.uniform(n)  # (0, 1]
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)

    def unit_vector(self, n: int = 1) -> np.ndarray:
        z = self.uniform(n, -1.0, 1.0)
        phi = self.uniform(n, 0.0, 2.0 * math.pi)
        r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=-1)

    def rotation(self) -> np.ndarray:
        """Uniform random rotation (Shoemake's quaternion method)."""
        u1, u2, u3 = self.uniform(3)
        a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
        x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
        z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
        return np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])


# ----------------------------------------------------------------------------
# Cameras (pinhole, OpenCV axes: x right, y down, z forward)
# ----------------------------------------------------------------------------
CAMERA_DTYPE = np.dtype([
    ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("width", "<i4"), ("height", "<i4"),
    ("R_cw", "<f4", (9,)), ("C", "<f4", (3,)),
])  # byte layout of the C struct otf_camera (72 bytes)
assert CAMERA_DTYPE.itemsize == 72

def _dot(a, b):
    """Row-wise dot product of (..., 3) arrays (or with a 3-vector), fixed order."""
    return a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1] + a[..., 2] * b[..., 2]


def _mat(v, M):
    """v @ M for (..., 3) rows v and a 3x3 M, written out."""
    return np.stack([v[..., 0] * M[0, j] + v[..., 1] * M[1, j] + v[..., 2] * M[2, j] for j in range(3)], axis=-1)


CENTRE = np.array([0.5, 0.5, 0.5])


def look_at(C: np.ndarray, target: np.ndarray = CENTRE) -> np.ndarray:
    """Camera->world rotation whose columns are the camera axes in world space."""
    fwd = target - C
    fwd = fwd / math.sqrt(float(_dot(fwd, fwd)))
    up = np.array([0.0, 0.0, 1.0])
    if abs(fwd[2]) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= math.sqrt(float(_dot(right, right)))
    down = np.cross(fwd, right)
    return np.stack([right, down, fwd], axis=1)


def make_camera(C, f: float, width: int, height: int, target=CENTRE) -> np.ndarray:
    cam = np.zeros((), dtype=CAMERA_DTYPE)
    R = look_at(np.asarray(C, dtype=np.float64), np.asarray(target, dtype=np.float64))
    cam["fx"] = cam["fy"] = f
    cam["cx"], cam["cy"] = width / 2.0, height / 2.0
    cam["width"], cam["height"] = width, height
    cam["R_cw"] = R.reshape(-1)
    cam["C"] = C
    return cam


def camera_rays(cam: np.ndarray):
    """Unit world-space directions of every pixel-centre ray, shape (H*W, 3)."""
    H, W = int(cam["height"]), int(cam["width"])
    jj, ii = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    dc = np.stack([(ii + 0.5 - float(cam["cx"])) / float(cam["fx"]),
                   (jj + 0.5 - float(cam["cy"])) / float(cam["fy"]),
                   np.ones_like(ii)], axis=-1).reshape(-1, 3)
    dc /= np.sqrt(_dot(dc, dc))[:, None]
    R = cam["R_cw"].astype(np.float64).reshape(3, 3)
    return np.asarray(cam["C"], dtype=np.float64), _mat(dc, R.T)


# ----------------------------------------------------------------------------
# Analytic primitives. intersect(o, d) returns the smallest t > 0 at which the
# ray o + t d meets the solid's boundary (inf if none). The camera is always
# outside every solid, so that point is where the ray enters the solid.
# ----------------------------------------------------------------------------
def _nearest(*cands):
    best = None
    for t, ok in cands:
        t = np.where(ok & (t > 1e-12), t, np.inf)
        best = t if best is None else np.minimum(best, t)
    return best


def _sphere_roots(o, d, c, r):
    oc = o - c
    b = _dot(d, oc)
    cc = _dot(oc, oc) - r * r
    disc = b * b - cc
    ok = disc >= 0
    s = np.sqrt(np.where(ok, disc, 0.0))
    return -b - s, -b + s, ok


@dataclass
class Sphere:
    c: np.ndarray
    r: float

    def intersect(self, o, d):
        t0, t1, ok = _sphere_roots(o, d, self.c, self.r)
        return _nearest((t0, ok), (t1, ok))


@dataclass
class Box:
    """Oriented box: centre c, rotation Q (columns = box axes), half-extents e."""
    c: np.ndarray
    Q: np.ndarray
    e: np.ndarray

    def intersect(self, o, d):
        ol = _mat(o - self.c, self.Q)
        dl = _mat(d, self.Q)
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-self.e - ol) / dl
            t2 = (self.e - ol) / dl
        tn = np.nanmax(np.minimum(t1, t2), axis=1)
        tf = np.nanmin(np.maximum(t1, t2), axis=1)
        hit = tn <= tf
        return _nearest((tn, hit), (tf, hit))


@dataclass
class Cylinder:
    """Capped cylinder: centre c, unit axis a, radius r, half-length hl."""
    c: np.ndarray
    a: np.ndarray
    r: float
    hl: float

    def intersect(self, o, d):
        oc = o - self.c
        da = _dot(d, self.a)
        oa = float(_dot(oc, self.a))
        dp = d - da[:, None] * self.a[None, :]
        op = oc - oa * self.a
        A = _dot(dp, dp)
        B = _dot(dp, op)
        Cc = float(_dot(op, op)) - self.r * self.r
        disc = B * B - A * Cc
        ok = (disc >= 0) & (A > 1e-300)
        s = np.sqrt(np.where(ok, disc, 0.0))
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (-B - s) / A
            tb = (-B + s) / A
            cands = []
            for t in (ta, tb):
                cands.append((t, ok & (np.abs(oa + t * da) <= self.hl)))
            for sgn in (-1.0, 1.0):
                t = (sgn * self.hl - oa) / da
                q = op + t[:, None] * dp
                cands.append((t, np.isfinite(t) & (_dot(q, q) <= self.r * self.r)))
        return _nearest(*cands)


@dataclass
class HemiShell:
    """Open spherical shell {ri <= |x - c| <= ro, (x - c) . n >= 0}."""
    c: np.ndarray
    ro: float
    ri: float
    n: np.ndarray

    def intersect(self, o, d):
        oc = o - self.c
        ocn = float(_dot(oc, self.n))
        dn = _dot(d, self.n)
        cands = []
        for r in (self.ro, self.ri):
            t0, t1, ok = _sphere_roots(o, d, self.c, r)
            for t in (t0, t1):
                side = ocn + t * dn
                cands.append((t, ok & (side >= 0)))
        with np.errstate(divide="ignore", invalid="ignore"):
            t = -ocn / dn
            q = oc + t[:, None] * d
            rr = _dot(q, q)
        cands.append((t, np.isfinite(t) & (rr >= self.ri ** 2) & (rr <= self.ro ** 2)))
        return _nearest(*cands)


def render(prims, cam) -> np.ndarray:
    """Radial range along every pixel-centre ray (0 where nothing is hit)."""
    o, d = camera_rays(cam)
    t = np.full(d.shape[0], np.inf)
    for p in prims:
        t = np.minimum(t, p.intersect(o, d))
    t = np.where(np.isfinite(t), t, 0.0)
    return t.reshape(int(cam["height"]), int(cam["width"]))


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
TAU_STEP = float(np.float32(1.0 / math.sqrt(12.0)))  # primal and dual step, tau*sigma*12 = 1


@dataclass
class Workload:
    name: str
    max_depth: int
    depth: np.ndarray          # (n_views, H, W) float32 radial range, 0 = invalid
    cams: np.ndarray           # (n_views,) CAMERA_DTYPE
    params: dict               # construction / restructure parameters (world units)
    iterations: int
    lam: float = 0.5
    tau: float = TAU_STEP
    sigma: float = TAU_STEP
    prims: list = field(default_factory=list)


def default_params(max_depth: int, delta_voxels: float, **over) -> dict:
    h = 2.0 ** -max_depth
    p = dict(max_depth=max_depth, delta=delta_voxels * h, eta=10.0 * delta_voxels * h,
             spread_tau=0.1, gamma=1e-2, split_tau=0.5, join_tau=0.9,
             restructure_every=1, max_leaves=0)
    p.update(over)
    return p


def _circle_cams(n, radius, f, W, H):
    cams = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        C = CENTRE + radius * np.array([math.cos(a), math.sin(a), 0.0])
        cams.append(make_camera(C, f, W, H))
    return np.array(cams, dtype=CAMERA_DTYPE)


def _hemisphere_cams(rng: Stream, n, radius, f, W, H):
    cams = []
    for _ in range(n):
        z = rng.uniform(1, 0.1, 0.95)[0]
        phi = rng.uniform(1, 0.0, 2.0 * math.pi)[0]
        r = math.sqrt(1.0 - z * z)
        C = CENTRE + radius * np.array([r * math.cos(phi), r * math.sin(phi), z])
        cams.append(make_camera(C, f, W, H))
    return np.array(cams, dtype=CAMERA_DTYPE)


def _render_all(prims, cams, noise):
    """Render and perturb every view (views in parallel threads; each view's
    result depends only on its own camera and random streams)."""
    import concurrent.futures as cf
    import os

    out = np.zeros((len(cams), int(cams[0]["height"]), int(cams[0]["width"])), dtype=np.float32)

    def one(i):
        out[i] = noise(i, cams[i], render(prims, cams[i])).astype(np.float32)

    workers = max(1, min(16, os.cpu_count() or 1, len(cams)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(one, range(len(cams))))
    return out


def sphere_workload(seed: int = 0, max_depth: int = 6, n_views: int = 8, W: int = 160, H: int = 120,
                    f: float = 150.0, radius: float = 0.3, centre=CENTRE, cam_radius: float = 1.2,
                    rel_noise: float = 0.005, delta_voxels: float = 3.0, iterations: int = 200,
                    workload_id: int = 1, **param_over) -> Workload:
    """A sphere seen from n_views poses on the circle z = 0.5 (the sphere stand-in)."""
    prims = [Sphere(np.asarray(centre, dtype=np.float64), radius)]
    cams = _circle_cams(n_views, cam_radius, f, W, H)

    def noise(i, cam, D):
        if rel_noise <= 0:
            return D
        n = Stream(workload_id, seed, 100 + i).normal(D.size).reshape(D.shape)
        return np.where(D > 0, D * (1.0 + rel_noise * n), 0.0)

    depth = _render_all(prims, cams, noise)
    return Workload("sphere", max_depth, depth, cams, default_params(max_depth, delta_voxels, **param_over),
                    iterations, prims=prims)


def blocks_workload(seed: int = 0, max_depth: int = 8, n_views: int = 32, W: int = 640, H: int = 480,
                    f: float = 600.0, iterations: int = 500, **param_over) -> Workload:
    """Union of 6 random spheres and 4 random oriented boxes, hemisphere poses,
    additive noise of one finest voxel plus 2% uniform outlier pixels."""
    wid = 2
    rng = Stream(wid, seed, 0)
    h = 2.0 ** -max_depth
    prims = []
    for _ in range(6):
        prims.append(Sphere(rng.uniform(3, 0.25, 0.75), float(rng.uniform(1, 0.05, 0.20)[0])))
    for _ in range(4):
        c = rng.uniform(3, 0.25, 0.75)
        e = rng.uniform(3, 0.03, 0.15)
        prims.append(Box(c, rng.rotation(), e))
    cams = _hemisphere_cams(Stream(wid, seed, 1), n_views, 1.6, f, W, H)

    def noise(i, cam, D):
        n = Stream(wid, seed, 100 + i).normal(D.size).reshape(D.shape)
        D = np.where(D > 0, D + h * n, 0.0)
        s = Stream(wid, seed, 200 + i)
        out = s.uniform(D.size).reshape(D.shape) < 0.02
        dc = np.asarray(cam["C"], dtype=np.float64) - CENTRE
        R = math.sqrt(float(_dot(dc, dc)))
        val = s.uniform(D.size, R - math.sqrt(3) / 2, R + math.sqrt(3) / 2).reshape(D.shape)
        return np.where(out, val, D)

    depth = _render_all(prims, cams, noise)
    return Workload("blocks", max_depth, depth, cams, default_params(max_depth, 4.0, **param_over),
                    iterations, prims=prims)


def thin_workload(seed: int = 0, max_depth: int = 9, n_views: int = 64, W: int = 640, H: int = 480,
                  f: float = 600.0, iterations: int = 1000, **param_over) -> Workload:
    """Thin structures: 3 slabs, 6 capped cylinders of radius 2-6 finest voxels and
    3 open hemispherical shells, hemisphere poses, 0.5% multiplicative noise."""
    wid = 3
    rng = Stream(wid, seed, 0)
    h = 2.0 ** -max_depth
    prims = []
    for _ in range(3):
        c = rng.uniform(3, 0.25, 0.75)
        lat = rng.uniform(2, 0.2, 0.45)
        th = float(rng.uniform(1, 2.0, 6.0)[0]) * h
        prims.append(Box(c, rng.rotation(), np.array([lat[0], lat[1], th / 2.0])))
    for _ in range(6):
        c = rng.uniform(3, 0.25, 0.75)
        r = float(rng.uniform(1, 2.0, 6.0)[0]) * h
        ln = float(rng.uniform(1, 0.3, 0.8)[0])
        prims.append(Cylinder(c, rng.unit_vector(1)[0], r, ln / 2.0))
    for _ in range(3):
        c = rng.uniform(3, 0.25, 0.75)
        ro = float(rng.uniform(1, 0.1, 0.3)[0])
        th = float(rng.uniform(1, 2.0, 6.0)[0]) * h
        prims.append(HemiShell(c, ro, ro - th, rng.unit_vector(1)[0]))
    cams = _hemisphere_cams(Stream(wid, seed, 1), n_views, 1.6, f, W, H)

    def noise(i, cam, D):
        n = Stream(wid, seed, 100 + i).normal(D.size).reshape(D.shape)
        return np.where(D > 0, D * (1.0 + 0.005 * n), 0.0)

    depth = _render_all(prims, cams, noise)
    return Workload("thin", max_depth, depth, cams, default_params(max_depth, 3.0, **param_over),
                    iterations, prims=prims)


def batch_workloads(n_objects: int = 48, first_seed: int = 1000, restructure_every: int = 0) -> list:
    """Many independent sphere objects (the batched workload): object j draws
    its max depth uniformly from {6, 7, 8, 9} and its view count from
    {8, ..., 64} with seed first_seed + j, views on the circle as in the sphere
    workload (160x120, f = 150)."""
    out = []
    for j in range(n_objects):
        s = Stream(4, first_seed + j, 0)
        D = 6 + int(s.uniform(1)[0] * 4)
        V = 8 + int(s.uniform(1)[0] * 57)
        w = sphere_workload(seed=first_seed + j, max_depth=D, n_views=V, workload_id=4,
                            restructure_every=restructure_every)
        w.name = f"batch-object-{j}"
        out.append(w)
    return out


def warm_training_workload(j: int, restructure_every: int = 0) -> Workload:
    """Training scene j of the learned warm start: a sphere as in the sphere
    workload with radius uniform in [0.2, 0.35] and its centre moved by up to
    0.05 per axis (seed j)."""
    s = Stream(5, j, 0)
    r = float(s.uniform(1, 0.2, 0.35)[0])
    c = CENTRE + s.uniform(3, -0.05, 0.05)
    w = sphere_workload(seed=j, radius=r, centre=c, workload_id=5, restructure_every=restructure_every)
    w.name = f"warm-train-{j}"
    return w


def workload(k: int, seed: int = 0, **kw) -> Workload:
    """The three plain-method workloads: 1 sphere (depth 6), 2 blocks (depth 8), 3 thin (depth 9)."""
    if k == 1:
        return sphere_workload(seed=seed, **kw)
    if k == 2:
        return blocks_workload(seed=seed, **kw)
    if k == 3:
        return thin_workload(seed=seed, **kw)
    raise ValueError(f"unknown workload {k}")


# ----------------------------------------------------------------------------
# Per-voxel volumes for tests that bypass the depth maps
# ----------------------------------------------------------------------------
def random_volumes(n_views: int, max_depth: int, seed: int, p_unobserved: float = 0.0,
                   smooth: bool = True, workload_id: int = 90):
    """Random per-view finest-voxel values f in [-1, 1] and observation masks w.

    With smooth=True the values come from a signed distance to a random plane
    through the volume plus noise, so that octree construction produces an
    unbalanced tree instead of a full refinement everywhere.
    """
    G = 1 << max_depth
    s = Stream(workload_id, seed, 0)
    f = np.empty((n_views, G, G, G), dtype=np.float32)  # index [v, z, y, x]
    w = np.empty((n_views, G, G, G), dtype=np.uint8)
    zz, yy, xx = np.meshgrid(*(np.arange(G) + 0.5,) * 3, indexing="ij")
    for v in range(n_views):
        if smooth:
            nrm = s.unit_vector(1)[0]
            c = s.uniform(3, 0.3, 0.7) * G
            width = float(s.uniform(1, 1.0, 3.0)[0])
            dist = (xx - c[0]) * nrm[0] + (yy - c[1]) * nrm[1] + (zz - c[2]) * nrm[2]
            val = np.clip(dist / width, -1.0, 1.0) + 0.05 * s.normal(G ** 3).reshape(G, G, G)
            f[v] = np.clip(val, -1.0, 1.0)
        else:
            f[v] = s.uniform(G ** 3, -1.0, 1.0).reshape(G, G, G)
        w[v] = (s.uniform(G ** 3) >= p_unobserved).reshape(G, G, G)
    return f, w
