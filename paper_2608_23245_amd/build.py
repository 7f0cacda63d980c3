"""Build the gfx950 HIP library libfdtbx.so in-tree (hipcc, no JIT cache).

Every translation unit is compiled for gfx950 only, with packed-FP32 code
generation disabled.  exact.hip (enumeration, pixel map, culling records and
lists), splat.hip (sample positions and their detector pixels), cyl.hip (ring
quadrature sizes) and points.hip (the Ewald projection) are compiled without
floating-point contraction so that their binary64 predicates are
evaluated exactly as written.

The example program examples/fdtbx_pattern.cpp, a caller of the C ABI without Python, is
linked against the library as _lib/fdtbx_pattern (run path $ORIGIN).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libfdtbx.so")
EXAMPLE = os.path.join(OUT_DIR, "fdtbx_pattern")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = {
    "exact.hip": ["-ffp-contract=off"],
    "nodes.hip": [],
    "sf.hip": [],
    "profile.hip": [],
    "adjoint.hip": [],
    "splat.hip": ["-ffp-contract=off"],
    "cyl.hip": ["-ffp-contract=off"],
    "points.hip": ["-ffp-contract=off"],
    "order.hip": [],
    "pairs.hip": [],
    "capi.hip": [],
}

COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        cmd = [cc, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    tmp = EXAMPLE + ".tmp"
    cmd = [cc, *COMMON, "-I", INCLUDE, os.path.join(HERE, "examples", "fdtbx_pattern.cpp"), "-o", tmp,
           "-L", OUT_DIR, "-lfdtbx", "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, EXAMPLE)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
