"""The C-ABI library loads and exports every entry point the header declares
(no compute calls: CPU only)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "otf.h")
LIB = os.path.join(ROOT, "paper_1608_07411_amd", "lib", "libotf.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:otf_status|const char \*)\s*(otf_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("otf_create", "otf_destroy", "otf_build_octree", "otf_fuse", "otf_extract", "otf_num_leaves",
                 "otf_energy", "otf_export_state", "otf_import_state", "otf_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libotf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1608_07411_amd import otf
    with pytest.raises(OSError):
        otf.lib(str(tmp_path / "missing.so"))
    with pytest.raises(OSError):
        otf.Context(0, library=str(tmp_path / "missing.so"))


def test_record_layouts():
    from paper_1608_07411_amd import otf, synth
    assert synth.CAMERA_DTYPE.itemsize == 72
    assert otf.PARAMS_DTYPE.itemsize == 40
    import oracle
    assert oracle.PARAMS_DTYPE == otf.PARAMS_DTYPE
    assert otf.ITER_RECORD_DTYPE.itemsize == 48


@pytest.mark.skipif(not os.path.exists(LIB), reason="libotf.so not built")
def test_null_context_is_invalid_before_any_device_work():
    """Entry points validate their arguments before any device call: a null
    context (or network) returns OTF_E_INVALID (1) on a machine without a GPU."""
    from paper_1608_07411_amd import otf
    L = otf.lib()
    calls = {
        "otf_fuse": (None, 1, 0.5, 0.3, 0.3),
        "otf_fuse_gd": (None, 1, 0.5, 0.1, 0.3),
        "otf_num_leaves": (None, None),
        "otf_energy": (None, None, None),
        "otf_extract": (None, 0, None, None, None, None, None, None),
        "otf_extract_obs_at": (None, 0, None, None, None, None, 0, None, None, None),
        "otf_obs_pool_stats": (None, None, None, None),
        "otf_warm_start": (None, None),
        "otf_warm_start_guarded": (None, None, 0.5, 1, None, None, None),
        "otf_export_state": (None, None, 0, None),
        "otf_selftest_scan": (None, 0, 0, None),
        "otf_debug_poke_guard": (None,),
        "otf_debug_unwritten_slot": (None,),
        "otf_log_every": (None, 1, None, 0),
        "otf_log_count": (None, None),
    }
    for name, args in calls.items():
        assert getattr(L, name)(*args) == 1, name


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; more is refused with a message (exit 2)
    before anything touches a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
