"""ctypes wrapper of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIBDIR, build

PARAMS_DTYPE = np.dtype([
    ("max_depth", "<i4"), ("delta", "<f4"), ("eta", "<f4"), ("spread_tau", "<f4"),
    ("gamma", "<f4"), ("split_tau", "<f4"), ("join_tau", "<f4"),
    ("restructure_every", "<i4"), ("max_leaves", "<i8"),
])
assert PARAMS_DTYPE.itemsize == 40

_LIBS: dict = {}


def _lib(precision: str):
    if precision not in _LIBS:
        path = os.path.join(LIBDIR, f"liboracle_{precision}.so")
        if not os.path.exists(path):
            build()
        lib = C.CDLL(path)
        P = C.c_void_p
        lib.orc_create.restype = P
        lib.orc_destroy.argtypes = [P]
        lib.orc_last_error.restype = C.c_char_p
        lib.orc_last_error.argtypes = [P]
        lib.orc_build.argtypes = [P, P, C.c_int, P, P]
        lib.orc_build_volumes.argtypes = [P, P, P, C.c_int, P]
        lib.orc_tsdf_volume.argtypes = [P, C.c_int, P, P, C.c_int, P, P]
        lib.orc_fuse.argtypes = [P, C.c_int, C.c_float, C.c_float, C.c_float]
        lib.orc_fuse_gd.argtypes = [P, C.c_int, C.c_float, C.c_float, C.c_float]
        lib.orc_energy_eps.argtypes = [P, C.c_double, P, P]
        lib.orc_num_leaves.restype = C.c_int64
        lib.orc_num_leaves.argtypes = [P]
        lib.orc_last_counts.argtypes = [P, P, P]
        lib.orc_extract.argtypes = [P, C.c_int64, P, P, P, P, P]
        lib.orc_num_obs.restype = C.c_int64
        lib.orc_num_obs.argtypes = [P]
        lib.orc_leaf_obs.argtypes = [P, P, P, P, P, P]
        lib.orc_neighbours.restype = C.c_int64
        lib.orc_neighbours.argtypes = [P, P, C.c_int64, P]
        lib.orc_apply_grad.argtypes = [P, P, P]
        lib.orc_apply_div.argtypes = [P, P, P]
        lib.orc_energy.argtypes = [P, P, P]
        lib.orc_prox.restype = C.c_double
        lib.orc_prox.argtypes = [C.c_int, P, P, C.c_double, C.c_double, C.c_double]
        lib.orc_export_state.argtypes = [P, P, C.c_int64, P]
        lib.orc_restructure_now.argtypes = [P, C.c_float, C.c_float]
        lib.orc_extract_aux.argtypes = [P, C.c_int64, P, P, P]
        lib.orc_import_state.argtypes = [P, P, C.c_int64]
        _LIBS[precision] = lib
    return _LIBS[precision]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def params_record(p: dict) -> np.ndarray:
    r = np.zeros((), dtype=PARAMS_DTYPE)
    for k in PARAMS_DTYPE.names:
        r[k] = p.get(k, 0)
    return r


class OracleError(RuntimeError):
    pass


class Oracle:
    """One fused octree on the CPU. precision: 'f32' (canonical, for bit parity)
    or 'f64' (for the self-checks)."""

    def __init__(self, precision: str = "f64"):
        self.lib = _lib(precision)
        self.precision = precision
        self.h = self.lib.orc_create()
        self.max_depth = None

    def __del__(self):
        try:
            self.lib.orc_destroy(self.h)
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise OracleError(f"oracle status {st}: {self.lib.orc_last_error(self.h).decode()}")

    # construction ------------------------------------------------------
    def build(self, depth: np.ndarray, cams: np.ndarray, params: dict):
        depth = np.ascontiguousarray(depth, dtype=np.float32)
        cams = np.ascontiguousarray(cams)
        prm = params_record(params)
        self._check(self.lib.orc_build(self.h, _ptr(depth), int(depth.shape[0]), _ptr(cams), _ptr(prm)))
        self.max_depth = int(params["max_depth"])
        return self

    def build_volumes(self, f: np.ndarray, w: np.ndarray, params: dict):
        f = np.ascontiguousarray(f, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.uint8)
        prm = params_record(params)
        self._check(self.lib.orc_build_volumes(self.h, _ptr(f), _ptr(w), int(f.shape[0]), _ptr(prm)))
        self.max_depth = int(params["max_depth"])
        return self

    def import_state(self, blob: bytes):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        self._check(self.lib.orc_import_state(self.h, _ptr(buf), buf.size))
        self.max_depth = int(np.frombuffer(blob[8:12], dtype="<i4")[0])
        return self

    def export_state(self) -> bytes:
        n = C.c_int64(0)
        self.lib.orc_export_state(self.h, None, 0, C.byref(n))
        buf = np.zeros(n.value, dtype=np.uint8)
        self._check(self.lib.orc_export_state(self.h, _ptr(buf), buf.size, C.byref(n)))
        return buf.tobytes()

    # solver --------------------------------------------------------------
    def fuse(self, iterations: int, lam: float, tau: float, sigma: float):
        self._check(self.lib.orc_fuse(self.h, int(iterations), lam, tau, sigma))
        return self

    def fuse_gd(self, iterations: int, lam: float, xi: float, eps: float):
        """The paper's gradient descent (lambda on TV, step xi, smoothing eps)."""
        self._check(self.lib.orc_fuse_gd(self.h, int(iterations), lam, xi, eps))
        return self

    def restructure_now(self, lam: float, tau: float):
        """Split/join of the current state, as the fuse loop runs it after an
        iteration's primal phase (test hook: only right after a fuse whose last
        iteration did not restructure)."""
        self._check(self.lib.orc_restructure_now(self.h, lam, tau))
        return self

    def extract_aux(self) -> dict:
        """Per leaf: u' and u_old of the last primal step or split cascade, and
        the split flag."""
        n = self.num_leaves()
        up = np.zeros(n)
        uo = np.zeros(n)
        sp = np.zeros(n, np.int32)
        self._check(self.lib.orc_extract_aux(self.h, n, _ptr(up), _ptr(uo), _ptr(sp)))
        return dict(uprime=up, uold=uo, split=sp.astype(bool))

    def last_counts(self):
        s, j = C.c_int64(0), C.c_int64(0)
        self.lib.orc_last_counts(self.h, C.byref(s), C.byref(j))
        return s.value, j.value

    def num_leaves(self) -> int:
        return int(self.lib.orc_num_leaves(self.h))

    def extract(self) -> dict:
        n = self.num_leaves()
        keys = np.zeros(n, np.uint32)
        levels = np.zeros(n, np.uint8)
        u = np.zeros(n)
        ubar = np.zeros(n)
        p = np.zeros((n, 3))
        self._check(self.lib.orc_extract(self.h, n, _ptr(keys), _ptr(levels), _ptr(u), _ptr(ubar), _ptr(p)))
        return dict(keys=keys, levels=levels, u=u, ubar=ubar, p=p)

    def leaf_obs(self) -> dict:
        n = self.num_leaves()
        m = int(self.lib.orc_num_obs(self.h))
        M = np.zeros(n, np.int32)
        wtot = np.zeros(n)
        inv = np.zeros(n)
        F = np.zeros(max(m, 1))
        W = np.zeros(max(m, 1))
        self._check(self.lib.orc_leaf_obs(self.h, _ptr(M), _ptr(wtot), _ptr(inv), _ptr(F), _ptr(W)))
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(M)
        return dict(M=M, wtot=wtot, inv=inv, F=F[:m], W=W[:m], off=off)

    def neighbours(self):
        """counts (L, 6) for faces +x,+y,+z,-x,-y,-z and concatenated indices."""
        n = self.num_leaves()
        counts = np.zeros((n, 6), np.int32)
        tot = int(self.lib.orc_neighbours(self.h, _ptr(counts), 0, None))
        idx = np.zeros(max(tot, 1), np.int64)
        self.lib.orc_neighbours(self.h, _ptr(counts), tot, _ptr(idx))
        return counts, idx[:tot]

    def grad(self, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        g = np.zeros((u.size, 3))
        self._check(self.lib.orc_apply_grad(self.h, _ptr(u), _ptr(g)))
        return g

    def div(self, p: np.ndarray) -> np.ndarray:
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(p.shape[0])
        self._check(self.lib.orc_apply_div(self.h, _ptr(p), _ptr(out)))
        return out

    def energy(self):
        tv, data = C.c_double(0), C.c_double(0)
        self._check(self.lib.orc_energy(self.h, C.byref(tv), C.byref(data)))
        return tv.value, data.value

    def energy_eps(self, eps: float):
        """Smoothed terms (tv, data) of the gradient-descent energy."""
        tv, data = C.c_double(0), C.c_double(0)
        self._check(self.lib.orc_energy_eps(self.h, float(eps), C.byref(tv), C.byref(data)))
        return tv.value, data.value


def prox(F, W, gamma: float, uprime: float, tl: float, precision: str = "f64") -> float:
    """Standalone generalised-shrinkage prox on unsorted observations."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    return float(_lib(precision).orc_prox(int(F.size), _ptr(F), _ptr(W), gamma, uprime, tl))


def tsdf_volume(depth, cams, params, view: int, precision: str = "f64"):
    """Eq. 1 evaluated at every finest voxel of one view: (f, w), index [z, y, x]."""
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    cams = np.ascontiguousarray(cams)
    G = 1 << int(params["max_depth"])
    f = np.zeros((G, G, G))
    w = np.zeros((G, G, G), np.uint8)
    prm = params_record(params)
    st = _lib(precision).orc_tsdf_volume(_ptr(depth), int(depth.shape[0]), _ptr(cams), _ptr(prm), view,
                                         _ptr(f), _ptr(w))
    if st:
        raise OracleError(f"tsdf_volume status {st}")
    return f, w


def morton_decode(keys: np.ndarray):
    keys = np.asarray(keys, dtype=np.uint64)
    x = np.zeros_like(keys)
    y = np.zeros_like(keys)
    z = np.zeros_like(keys)
    for b in range(10):
        x |= ((keys >> np.uint64(3 * b)) & np.uint64(1)) << np.uint64(b)
        y |= ((keys >> np.uint64(3 * b + 1)) & np.uint64(1)) << np.uint64(b)
        z |= ((keys >> np.uint64(3 * b + 2)) & np.uint64(1)) << np.uint64(b)
    return x.astype(np.int64), y.astype(np.int64), z.astype(np.int64)
