"""FP64 operation count of the cache build's local physics.

Builds `opcount.cpp` (the library's physics.h compiled on the host with a
counting scalar type) with g++ and runs it on the given classes: mean flops
(add, subtract, multiply, divide, square root) and transcendental calls per
energy evaluation and per theta_I solve, per kernel and mode.  The counts
follow the kernel source, so they change when physics.h does."""
from __future__ import annotations

import json
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)


def count(classes, n_dirs=360, n_sweep=1440, mode=1, kernel=0, start_offset=(1e-3, 2e-4)) -> dict:
    """classes: [K][13] chert_class rows.  Per (kernel, mode): flops and
    transcendental calls per energy evaluation and per theta_I solve; for
    `mode` and `kernel`, the build's steps per class: the n_sweep-sample
    theta_R sweep, the solve of each of the n_dirs / 2 directions, and the
    surrogate start's polish of each direction from its root offset by
    start_offset (theta_R, theta_I) [rad]."""
    rows = np.ascontiguousarray(np.atleast_2d(classes), dtype=np.float64)
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "opcount")
        cmd = ["g++", "-O1", "-std=c++20", "-ffp-contract=off", "-I", HERE,
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
               os.path.join(HERE, "opcount.cpp"), "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        text = "\n".join(" ".join(repr(float(x)) for x in r) for r in rows) + "\n"
        env = dict(os.environ, OPCOUNT_ARGS=f"{n_dirs} {n_sweep} {mode} {kernel} "
                                             f"{start_offset[0]!r} {start_offset[1]!r}")
        out = subprocess.run([exe], input=text, check=True, capture_output=True, text=True,
                             env=env)
    return json.loads(out.stdout)
