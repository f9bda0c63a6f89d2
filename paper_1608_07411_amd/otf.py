"""Thin ctypes binding of libotf (include/otf.h): argument marshalling only.

Every step of the fusion runs in the HIP library. PyTorch supplies the stream
(and, optionally, device memory for the range maps). Loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .synth import CAMERA_DTYPE

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libotf.so")
# the bounds-checked build (OTF_DEBUG_BOUNDS): every adjacency index and
# observation segment the sweeps read is checked on the device
BOUNDS_LIB_PATH = os.path.join(HERE, "lib", "libotf_bounds.so")

PARAMS_DTYPE = np.dtype([
    ("max_depth", "<i4"), ("delta", "<f4"), ("eta", "<f4"), ("spread_tau", "<f4"),
    ("gamma", "<f4"), ("split_tau", "<f4"), ("join_tau", "<f4"),
    ("restructure_every", "<i4"), ("max_leaves", "<i8"),
])

# otf_iter_record: one per logged iteration (otf_log_every)
ITER_RECORD_DTYPE = np.dtype([
    ("iteration", "<i8"), ("leaves", "<i8"), ("splits", "<i8"), ("joins", "<i8"), ("tv", "<f8"), ("data", "<f8"),
])

STATUS = {0: "OTF_OK", 1: "OTF_E_INVALID", 2: "OTF_E_NOMEM", 3: "OTF_E_CAPACITY", 4: "OTF_E_DEVICE",
          5: "OTF_E_STATE"}
PROFILE_KINDS = ("dual", "primal", "restructure", "energy")

_libs: dict = {}


class OtfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib(path: str = LIB_PATH):
    """Load libotf.so, or another build of it at `path` (raises if it was not built)."""
    if path not in _libs:
        if not os.path.exists(path):
            raise OSError(f"{os.path.basename(path)} not found at {path}; build it with "
                          f"paper_1608_07411_amd.build.build()")
        # PyTorch, when present, brings its own HIP runtime library: load it
        # first, so that this library binds to the same runtime instead of
        # loading a second one into the process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(path)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "otf_create": [C.c_int, P, P],
            "otf_destroy": [P],
            "otf_build_octree": [P, P, I32, I32, P, P],
            "otf_fuse": [P, I32, C.c_float, C.c_float, C.c_float],
            "otf_fuse_graph_iterations": [P, P],
            "otf_num_leaves": [P, P],
            "otf_extract": [P, I64, P, P, P, P, P, P],
            "otf_extract_obs": [P, I64, P, P, P, I64, P, P, P],
            "otf_extract_neighbours": [P, I64, P, I64, P, P],
            "otf_energy": [P, P, P],
            "otf_energy_noalloc": [P, P, P],
            "otf_debug_fail_allocations": [P, C.c_int64],
            "otf_debug_corrupt_adjacency": [P, C.c_int64],
            "otf_debug_poke_guard": [P],
            "otf_debug_unwritten_slot": [P],
            "otf_log_every": [P, C.c_int32, P, C.c_int64],
            "otf_log_count": [P, P],
            "otf_fuse_gd": [P, I32, C.c_float, C.c_float, C.c_float],
            "otf_dense_field": [P, P, I32, I64],
            "otf_mesh": [P, C.c_float, I64, P, P, P],
            "otf_quantisation_error": [P, P, I32, P],
            "otf_mlp_create": [C.c_int, P, P],
            "otf_mlp_destroy": [P],
            "otf_mlp_set_params": [P, P, I64],
            "otf_mlp_get_params": [P, P, I64],
            "otf_mlp_forward": [P, P, I64, P],
            "otf_mlp_gradient": [P, P, P, I64, P, P],
            "otf_mlp_train_step": [P, P, P, I64, C.c_float, P],
            "otf_features": [P, P, I64],
            "otf_leaf_targets": [P, P, I64],
            "otf_warm_start": [P, P],
            "otf_warm_start_guarded": [P, P, C.c_float, I32, P, P, P],
            "otf_energy_eps": [P, C.c_double, P, P],
            "otf_last_counts": [P, P, P],
            "otf_export_state": [P, P, I64, P],
            "otf_import_state": [P, P, I64],
            "otf_profile": [P, I32],
            "otf_profile_read": [P, P, P, P, P],
            "otf_profile_read_eval": [P, P, P],
            "otf_batch_create": [C.c_int, P, P],
            "otf_batch_destroy": [P],
            "otf_batch_add": [P, P],
            "otf_batch_fuse": [P, I32, C.c_float, C.c_float, C.c_float],
            "otf_batch_config": [P, P, P, P, P],
            "otf_selftest_scan": [P, I64, C.c_uint64, P],
            "otf_obs_pool_stats": [P, P, P, P],
            "otf_extract_obs_at": [P, I64, P, P, P, P, I64, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.otf_last_error.argtypes = [P]
        L.otf_last_error.restype = C.c_char_p
        L.otf_batch_last_error.argtypes = [P]
        L.otf_batch_last_error.restype = C.c_char_p
        L.otf_mlp_last_error.argtypes = [P]
        L.otf_mlp_last_error.restype = C.c_char_p
        L.otf_mlp_num_params.argtypes = []
        L.otf_mlp_num_params.restype = I64
        _libs[path] = L
    return _libs[path]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def params_record(p: dict) -> np.ndarray:
    r = np.zeros((), dtype=PARAMS_DTYPE)
    for k in PARAMS_DTYPE.names:
        r[k] = p.get(k, 0)
    return r


def _stream_handle(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    except Exception:
        pass
    return C.c_void_p(0)


def _host_arrays(*specs):
    """Host arrays of the given (shape, dtype) for device-to-host copies: in
    page-locked memory when torch has a GPU (a copy into pageable memory is
    staged by the runtime at a fraction of the rate), else plain numpy."""
    try:
        import torch
        if torch.cuda.is_available():
            out = []
            for shape, dt in specs:
                t = torch.empty(int(np.prod(shape)) * np.dtype(dt).itemsize, dtype=torch.uint8, pin_memory=True)
                out.append(t.numpy().view(dt).reshape(shape))
            return out
    except ImportError:
        pass
    return [np.empty(shape, dt) for shape, dt in specs]


class Context:
    """One fused octree on one GPU (otf_ctx)."""

    def __init__(self, device: int = 0, stream=None, library: str = LIB_PATH):
        self._lib = lib(library)
        self.h = C.c_void_p()
        self._D = None
        self._check(self._lib.otf_create(device, _stream_handle(stream), C.byref(self.h)), "otf_create")

    def close(self):
        if self.h:
            self._lib.otf_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            msg = self._lib.otf_last_error(self.h).decode() if self.h else what
            raise OtfError(st, f"{what}: {msg}")

    # construction -----------------------------------------------------------
    def build_octree(self, depth, cams: np.ndarray, params: dict):
        cams = np.ascontiguousarray(cams, dtype=CAMERA_DTYPE)
        prm = params_record(params)
        is_dev = 0
        keep = depth
        if hasattr(depth, "is_cuda"):  # torch tensor
            if depth.is_cuda:
                keep = depth.contiguous().float()
                ptr = C.c_void_p(keep.data_ptr())
                is_dev = 1
            else:
                keep = depth.contiguous().float().numpy()
                ptr = _ptr(keep)
        else:
            keep = np.ascontiguousarray(depth, dtype=np.float32)
            ptr = _ptr(keep)
        n_views = int(keep.shape[0])
        self._check(self._lib.otf_build_octree(self.h, ptr, is_dev, n_views, _ptr(cams), _ptr(prm)),
                    "otf_build_octree")
        self._D = int(prm["max_depth"])
        return self

    def import_state(self, blob: bytes):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        self._check(self._lib.otf_import_state(self.h, _ptr(buf), buf.size), "otf_import_state")
        self._D = int(np.frombuffer(blob, dtype="<i4", count=1, offset=8)[0])
        return self

    def export_state(self) -> bytes:
        n = C.c_int64(0)
        self._check(self._lib.otf_export_state(self.h, None, 0, C.byref(n)), "otf_export_state")
        buf = np.zeros(n.value, np.uint8)
        self._check(self._lib.otf_export_state(self.h, _ptr(buf), buf.size, C.byref(n)), "otf_export_state")
        return buf.tobytes()

    # solver -----------------------------------------------------------------
    def fuse(self, iterations: int, lam: float, tau: float, sigma: float):
        self._check(self._lib.otf_fuse(self.h, int(iterations), lam, tau, sigma), "otf_fuse")
        return self

    def graph_iterations(self) -> int:
        """Iterations of the last fuse call replayed from a recorded graph."""
        n = C.c_int64(0)
        self._check(self._lib.otf_fuse_graph_iterations(self.h, C.byref(n)), "otf_fuse_graph_iterations")
        return n.value

    def fuse_gd(self, iterations: int, lam: float, step: float, eps: float):
        """The paper's gradient descent (lambda on TV, step, smoothing eps)."""
        self._check(self._lib.otf_fuse_gd(self.h, int(iterations), lam, step, eps), "otf_fuse_gd")
        return self

    def energy_eps(self, eps: float):
        """Smoothed (tv, data) terms of the gradient-descent energy."""
        tv, data = C.c_double(0), C.c_double(0)
        self._check(self._lib.otf_energy_eps(self.h, float(eps), C.byref(tv), C.byref(data)), "otf_energy_eps")
        return tv.value, data.value

    def dense_field(self, out=None):
        """u on the finest grid as a (G, G, G) [z, y, x] float32 array (or into a
        contiguous CUDA float tensor `out`)."""
        G = 1 << self.max_depth()
        if out is not None and hasattr(out, "is_cuda") and out.is_cuda:
            self._check(self._lib.otf_dense_field(self.h, C.c_void_p(out.data_ptr()), 1, out.numel()),
                        "otf_dense_field")
            return out
        a = np.zeros((G, G, G), np.float32)
        self._check(self._lib.otf_dense_field(self.h, _ptr(a), 0, a.size), "otf_dense_field")
        return a

    def mesh(self, iso: float = 0.0):
        """Marching-cubes triangles: (T, 3, 3) float32 vertices and (T, 3) uint64 edge ids."""
        n = C.c_int64(0)
        st = self._lib.otf_mesh(self.h, iso, 0, None, None, C.byref(n))
        if st not in (0, 3):
            self._check(st, "otf_mesh")
        xyz, ed = _host_arrays(((max(n.value, 1), 3, 3), np.float32), ((max(n.value, 1), 3), np.uint64))
        if n.value > 0:
            self._check(self._lib.otf_mesh(self.h, iso, n.value, _ptr(xyz), _ptr(ed), C.byref(n)), "otf_mesh")
        return xyz[:n.value], ed[:n.value]

    def quantisation_error(self, dense) -> float:
        """Eq. 7 against a finest-grid field (numpy array or CUDA tensor)."""
        err = C.c_double(0)
        if hasattr(dense, "is_cuda") and dense.is_cuda:
            st = self._lib.otf_quantisation_error(self.h, C.c_void_p(dense.data_ptr()), 1, C.byref(err))
        else:
            d = np.ascontiguousarray(dense, dtype=np.float32)
            st = self._lib.otf_quantisation_error(self.h, _ptr(d), 0, C.byref(err))
        self._check(st, "otf_quantisation_error")
        return err.value

    def max_depth(self) -> int:
        if self._D is None:
            raise OtfError(5, "no octree built or imported")
        return self._D

    def features(self):
        """Warm-start features of every leaf: CUDA float tensor (L, 32)."""
        import torch
        X = torch.empty((self.num_leaves(), 32), dtype=torch.float32, device="cuda")
        self._check(self._lib.otf_features(self.h, C.c_void_p(X.data_ptr()), X.shape[0]), "otf_features")
        return X

    def targets(self):
        """Current (u, px, py, pz) of every leaf: CUDA float tensor (L, 4)."""
        import torch
        T = torch.empty((self.num_leaves(), 4), dtype=torch.float32, device="cuda")
        self._check(self._lib.otf_leaf_targets(self.h, C.c_void_p(T.data_ptr()), T.shape[0]), "otf_leaf_targets")
        return T

    def warm_start(self, net: "Mlp"):
        """Replace u (and ubar) and p of every leaf by the network's prediction."""
        self._check(self._lib.otf_warm_start(self.h, net.h), "otf_warm_start")
        return self

    def warm_start_guarded(self, net: "Mlp", lam: float, alphas=(1.0, 0.5, 0.25)):
        """The prediction applied at the step (alphas, or 0: the current state)
        whose energy tv + lam * data is lowest; returns (alpha, energy)."""
        a = (C.c_float * len(alphas))(*alphas)
        au, eu = C.c_float(0), C.c_double(0)
        self._check(self._lib.otf_warm_start_guarded(self.h, net.h, float(lam), len(alphas), a, C.byref(au),
                                                    C.byref(eu)), "otf_warm_start_guarded")
        return au.value, eu.value

    def obs_pool_stats(self) -> dict:
        """Observation pool entries in use and reserved, and compactions so far."""
        u, cap, k = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        self._check(self._lib.otf_obs_pool_stats(self.h, C.byref(u), C.byref(cap), C.byref(k)), "otf_obs_pool_stats")
        return dict(used=u.value, capacity=cap.value, compactions=k.value)

    def selftest_scan(self, n: int, seed: int = 0) -> int:
        """Device scans against host scans on n pseudo-random elements; the
        number of differing outputs."""
        bad = C.c_int64(0)
        self._check(self._lib.otf_selftest_scan(self.h, n, seed, C.byref(bad)), "otf_selftest_scan")
        return bad.value

    def num_leaves(self) -> int:
        n = C.c_int64(0)
        self._check(self._lib.otf_num_leaves(self.h, C.byref(n)), "otf_num_leaves")
        return n.value

    def last_counts(self):
        s, j = C.c_int64(0), C.c_int64(0)
        self._check(self._lib.otf_last_counts(self.h, C.byref(s), C.byref(j)), "otf_last_counts")
        return s.value, j.value

    def extract(self) -> dict:
        n = self.num_leaves()
        keys = np.zeros(n, np.uint32)
        levels = np.zeros(n, np.uint8)
        u = np.zeros(n, np.float32)
        ubar = np.zeros(n, np.float32)
        p = np.zeros((n, 3), np.float32)
        w = C.c_int64(0)
        self._check(self._lib.otf_extract(self.h, n, _ptr(keys), _ptr(levels), _ptr(u), _ptr(ubar), _ptr(p),
                                          C.byref(w)), "otf_extract")
        return dict(keys=keys, levels=levels, u=u, ubar=ubar, p=p)

    def extract_obs(self) -> dict:
        n = self.num_leaves()
        M = np.zeros(n, np.int32)
        wtot = np.zeros(n, np.float32)
        inv = np.zeros(n, np.float32)
        tot = C.c_int64(0)
        st = self._lib.otf_extract_obs(self.h, n, _ptr(M), _ptr(wtot), _ptr(inv), 0, None, None, C.byref(tot))
        if st not in (0, 3):
            self._check(st, "otf_extract_obs")
        F = np.zeros(max(tot.value, 1), np.float32)
        W = np.zeros(max(tot.value, 1), np.float32)
        self._check(self._lib.otf_extract_obs(self.h, n, _ptr(M), _ptr(wtot), _ptr(inv), F.size, _ptr(F), _ptr(W),
                                              C.byref(tot)), "otf_extract_obs")
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(M)
        return dict(M=M, wtot=wtot, inv=inv, F=F[:tot.value], W=W[:tot.value], off=off)

    def extract_obs_at(self, leaves) -> dict:
        """Observations of the listed leaves (indices in the current order)."""
        idx = np.ascontiguousarray(leaves, dtype=np.int64)
        n = idx.size
        M = np.zeros(n, np.int32)
        wtot = np.zeros(n, np.float32)
        inv = np.zeros(n, np.float32)
        tot = C.c_int64(0)
        self._check(self._lib.otf_extract_obs_at(self.h, n, _ptr(idx), _ptr(M), _ptr(wtot), _ptr(inv), 0, None, None,
                                                 C.byref(tot)), "otf_extract_obs_at")
        F = np.zeros(max(tot.value, 1), np.float32)
        W = np.zeros(max(tot.value, 1), np.float32)
        self._check(self._lib.otf_extract_obs_at(self.h, n, _ptr(idx), _ptr(M), _ptr(wtot), _ptr(inv), F.size,
                                                 _ptr(F), _ptr(W), C.byref(tot)), "otf_extract_obs_at")
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(M)
        return dict(M=M, wtot=wtot, inv=inv, F=F[:tot.value], W=W[:tot.value], off=off)

    def obs_counts(self) -> np.ndarray:
        """Observation count M of every leaf (no pool download)."""
        n = self.num_leaves()
        M = np.zeros(n, np.int32)
        tot = C.c_int64(0)
        self._check(self._lib.otf_extract_obs(self.h, n, _ptr(M), None, None, 0, None, None, C.byref(tot)),
                    "otf_extract_obs")
        return M

    def extract_neighbours(self):
        n = self.num_leaves()
        counts = np.zeros((n, 6), np.int32)
        tot = C.c_int64(0)
        st = self._lib.otf_extract_neighbours(self.h, n, _ptr(counts), 0, None, C.byref(tot))
        if st not in (0, 3):
            self._check(st, "otf_extract_neighbours")
        idx = np.zeros(max(tot.value, 1), np.int64)
        self._check(self._lib.otf_extract_neighbours(self.h, n, _ptr(counts), idx.size, _ptr(idx), C.byref(tot)),
                    "otf_extract_neighbours")
        return counts, idx[:tot.value]

    def energy(self):
        tv, data = C.c_double(0), C.c_double(0)
        self._check(self._lib.otf_energy(self.h, C.byref(tv), C.byref(data)), "otf_energy")
        return tv.value, data.value

    def debug_fail_allocations(self, after: int):
        """Test hook: the after-th later device allocation on this context fails (0: off)."""
        self._check(self._lib.otf_debug_fail_allocations(self.h, int(after)), "otf_debug_fail_allocations")

    def debug_corrupt_adjacency(self, leaf: int):
        """Test hook of the bounds-checked build: point leaf's first + entry past the last leaf."""
        self._check(self._lib.otf_debug_corrupt_adjacency(self.h, int(leaf)), "otf_debug_corrupt_adjacency")

    def log_every(self, k: int, capacity: int):
        """Arm the per-iteration log (every k-th iteration, up to capacity records)."""
        self._log = np.zeros(max(int(capacity), 0), ITER_RECORD_DTYPE)
        ptr = self._log.ctypes.data if self._log.size else None
        self._check(self._lib.otf_log_every(self.h, int(k), ptr, int(capacity)), "otf_log_every")
        return self

    def log(self):
        """The records written since log_every (a structured array)."""
        n = C.c_int64(0)
        self._check(self._lib.otf_log_count(self.h, C.byref(n)), "otf_log_count")
        return self._log[: n.value].copy()

    def debug_unwritten_slot(self):
        """Test hook of the bounds-checked build: the next neighbour search leaves + slot 0 unwritten."""
        self._check(self._lib.otf_debug_unwritten_slot(self.h), "otf_debug_unwritten_slot")

    def debug_poke_guard(self):
        """Test hook of the bounds-checked build: damage the guard zone after the + adjacency list."""
        self._check(self._lib.otf_debug_poke_guard(self.h), "otf_debug_poke_guard")

    def energy_noalloc(self):
        """otf_energy without device allocation (static library scratch)."""
        tv, data = C.c_double(0), C.c_double(0)
        self._check(self._lib.otf_energy_noalloc(self.h, C.byref(tv), C.byref(data)), "otf_energy_noalloc")
        return tv.value, data.value

    # profiling --------------------------------------------------------------
    def profile(self, enable: bool = True):
        self._check(self._lib.otf_profile(self.h, 1 if enable else 0), "otf_profile")

    def profile_read(self) -> dict:
        ms = np.zeros(4)
        n = np.zeros(4, np.int64)
        lu = C.c_int64(0)
        by = np.zeros(4)
        self._check(self._lib.otf_profile_read(self.h, _ptr(ms), _ptr(n), C.byref(lu), _ptr(by)), "otf_profile_read")
        out = {k: dict(ms=float(ms[i]), launches=int(n[i])) for i, k in enumerate(PROFILE_KINDS)}
        out["leaf_updates"] = lu.value
        out["bytes"] = dict(dual=float(by[0]), primal=float(by[1]))
        out["method_bytes"] = dict(dual=float(by[2]), primal=float(by[3]))
        return out

    def profile_read_eval(self) -> dict:
        """Event-timed evaluation kernels: field, eq7, mc_count, mc_emit."""
        ms = np.zeros(4)
        n = np.zeros(4, np.int64)
        self._check(self._lib.otf_profile_read_eval(self.h, _ptr(ms), _ptr(n)), "otf_profile_read_eval")
        return {k: dict(ms=float(ms[i]), launches=int(n[i]))
                for i, k in enumerate(("field", "eq7", "mc_count", "mc_emit"))}

    def reset_counters(self, profile: bool):
        """Zero the leaf-update and byte counters; enable or disable kernel timing."""
        self.profile(profile)


class Batch:
    """Many contexts swept by the same launches (otf_batch). Members stay owned
    by the caller and must outlive the batch."""

    def __init__(self, device: int = 0, stream=None, library: str = LIB_PATH):
        # members must come from the same build (library) as the batch
        self._lib = lib(library)
        self.h = C.c_void_p()
        self.members = []
        st = self._lib.otf_batch_create(device, _stream_handle(stream), C.byref(self.h))
        if st != 0:
            raise OtfError(st, "otf_batch_create")

    def close(self):
        if self.h:
            self._lib.otf_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise OtfError(st, f"{what}: {self._lib.otf_batch_last_error(self.h).decode()}")

    def add(self, ctx: Context):
        self._check(self._lib.otf_batch_add(self.h, ctx.h), "otf_batch_add")
        self.members.append(ctx)
        return self

    def fuse(self, iterations: int, lam: float, tau: float, sigma: float):
        self._check(self._lib.otf_batch_fuse(self.h, int(iterations), lam, tau, sigma), "otf_batch_fuse")
        return self

    def config(self) -> dict:
        b, g, t, gi = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
        self._check(self._lib.otf_batch_config(self.h, C.byref(b), C.byref(g), C.byref(t), C.byref(gi)),
                    "otf_batch_config")
        return dict(block=b.value, grid=g.value, tuned=bool(t.value), graph_iterations=gi.value)


class Mlp:
    """The warm-start network (otf_mlp): parameters, forward, gradient, Adam steps.
    X, T and Y are contiguous CUDA float tensors (rows x 32, rows x 4)."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = lib()
        self.h = C.c_void_p()
        st = self._lib.otf_mlp_create(device, _stream_handle(stream), C.byref(self.h))
        if st != 0:
            raise OtfError(st, "otf_mlp_create")
        self.n_params = int(self._lib.otf_mlp_num_params())

    def close(self):
        if self.h:
            self._lib.otf_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise OtfError(st, f"{what}: {self._lib.otf_mlp_last_error(self.h).decode()}")

    def set_params(self, theta: np.ndarray):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(self._lib.otf_mlp_set_params(self.h, _ptr(t), t.size), "otf_mlp_set_params")

    def get_params(self) -> np.ndarray:
        t = np.zeros(self.n_params, np.float32)
        self._check(self._lib.otf_mlp_get_params(self.h, _ptr(t), t.size), "otf_mlp_get_params")
        return t

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], 4), dtype=torch.float32, device=X.device)
        self._check(self._lib.otf_mlp_forward(self.h, C.c_void_p(X.data_ptr()), X.shape[0], C.c_void_p(Y.data_ptr())),
                    "otf_mlp_forward")
        return Y

    def gradient(self, X, T):
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_double(0)
        self._check(self._lib.otf_mlp_gradient(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                                X.shape[0], _ptr(g), C.byref(loss)), "otf_mlp_gradient")
        return loss.value, g

    def train_step(self, X, T, lr: float) -> float:
        loss = C.c_double(0)
        self._check(self._lib.otf_mlp_train_step(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                                  X.shape[0], lr, C.byref(loss)), "otf_mlp_train_step")
        return loss.value


def raw_status(fn_name: str, *args) -> int:
    """Call an entry point directly and return its status (tests of error paths)."""
    return getattr(lib(), fn_name)(*args)
