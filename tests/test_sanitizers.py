"""AddressSanitizer and UndefinedBehaviorSanitizer builds, CPU only:

* the oracle (plain C, gcc) driven through its whole C interface on small
  synthetic volumes (tests/native/oracle_driver.c), leak detection on;
* the library's host code (hipcc, sanitizers on the host side only) driven
  through the argument validation of every entry point
  (tests/native/abi_driver.cpp), which must reject bad calls before any
  device work.

Any sanitizer report fails the run (non-zero exit, report on stderr).
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1608_07411_amd", "csrc")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-mfma",
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(NATIVE, "oracle_driver.c"), "-o", exe,
                    "-lm"])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "oracle driver ok" in out and "Sanitizer" not in out, out


@pytest.mark.slow
def test_library_host_validation_under_asan_and_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_1608_07411_amd.build import HIPCC_FLAGS, SOURCES

    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    objs = []
    procs = []
    for src in SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, *HIPCC_FLAGS, *san, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, out
    lib = str(tmp_path / "libotf_san.so")
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *san, *objs, "-o", lib])
    assert rc == 0, out
    exe = str(tmp_path / "abi_driver")
    rc, out = _run([hipcc, "-std=c++17", "-O1", *san, f"-I{os.path.join(ROOT, 'include')}",
                    os.path.join(NATIVE, "abi_driver.cpp"), f"-L{tmp_path}", "-lotf_san", f"-Wl,-rpath,{tmp_path}",
                    "-o", exe])
    assert rc == 0, out
    # leaks inside the HIP runtime's own start-up are not this library's
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", LSAN_OPTIONS=f"suppressions={supp}",
               UBSAN_OPTIONS="print_stacktrace=1", HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    rc, out = _run([exe], env=env)
    assert rc == 0 and "abi driver ok" in out and "runtime error" not in out, out
    assert shutil.which("gcc")
