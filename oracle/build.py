"""Compile the CPU oracle (plain C) into two shared libraries: canonical fp32
and fp64. Test infrastructure only."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIBDIR = os.path.join(HERE, "lib")
FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-mfma",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> dict:
    os.makedirs(LIBDIR, exist_ok=True)
    src = os.path.join(HERE, "oracle.c")
    out = {}
    for name, extra in (("f32", ["-DORC_FP32"]), ("f64", [])):
        lib = os.path.join(LIBDIR, f"liboracle_{name}.so")
        tmp = lib + ".tmp"
        cmd = ["gcc", *FLAGS, *extra, src, "-o", tmp, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
        out[name] = lib
    return out


if __name__ == "__main__":
    build(verbose=True)
