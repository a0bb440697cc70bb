"""Build libchert.so (HIP, gfx950) in-tree with hipcc.

Per-file floating-point contraction:
  - cache_build.hip: FMA contraction allowed (the local solve is compared
    with a tolerance);
  - trace.hip, frontier.hip, tile3d.hip, cellnet.hip, abi_host.cpp:
    -ffp-contract=off, so edge weights, traveltime sums and the host-side
    star and segment lengths are plain IEEE operations.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libchert.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-result"]
SOURCES = [
    ("cache_build.hip", ["-ffp-contract=fast"]),
    ("trace.hip", ["-ffp-contract=off"]),
    ("frontier.hip", ["-ffp-contract=off"]),
    ("tile3d.hip", ["-ffp-contract=off"]),
    ("cellnet.hip", ["-ffp-contract=off"]),
    ("surrogate.hip", ["-ffp-contract=fast"]),
    ("abi_host.cpp", ["-ffp-contract=off", "-x", "hip"]),
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
