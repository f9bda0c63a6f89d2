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


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1608_07411_amd import otf
    monkeypatch.setattr(otf, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(otf, "_lib", None)
    with pytest.raises(OSError):
        otf.lib()


def test_record_layouts():
    from paper_1608_07411_amd import otf, synth
    assert synth.CAMERA_DTYPE.itemsize == 72
    assert otf.PARAMS_DTYPE.itemsize == 40
    import oracle
    assert oracle.PARAMS_DTYPE == otf.PARAMS_DTYPE
