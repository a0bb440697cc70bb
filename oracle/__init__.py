"""CHERT CPU oracle -- test infrastructure only.

A plain FP64 C implementation (``chert_oracle.c``) of what the CHERT hot path
computes, wrapped with ctypes.  Only the tests, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the HIP library (``paper_2609_26108_amd``) and neither imports
the other.

Every function cites the passage of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chert_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

QP, QSV, QSH = 0, 1, 2
MEV, OEV = 0, 1
ST_OK, ST_NO_BRACKET, ST_ILL, ST_FLUID, ST_NONPHYS, ST_NOCONV = 0, 1, 2, 4, 8, 16
FIELDS = ("V", "A", "Q", "rx", "rz", "thR", "thI", "res")
NF = len(FIELDS)
N_SWEEP = 1440

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with plain IEEE settings (no fast-math, no FMA)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        d, i, l, u = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_uint
        P = ctypes.c_void_p
        L.orc_thomsen.argtypes = [d, d, d, d, d, P]
        L.orc_velocity.argtypes = [P, i, i, d, d, P]
        L.orc_residual.argtypes = [P, i, i, d, d]
        L.orc_residual.restype = d
        L.orc_theta_imag.argtypes = [P, i, i, d, P]
        L.orc_solve.argtypes = [P, i, i, i, d, P]
        L.orc_sweep.argtypes = [P, i, i, i, P, P, P, P]
        L.orc_build_cache_2d.argtypes = [P, l, i, u, i, i, P, P]
        L.orc_build_cache_2d_cols.argtypes = [P, l, i, P, i, u, i, i, P, P]
        L.orc_trace_2d_cols.argtypes = [l, l, d, d, P, i, i, P, i, P, P, P, l,
                                        P, P, P, P, P, P, P]
        L.orc_star_2d.argtypes = [i, d, d, i, P, P, P, P]
        L.orc_trace_2d.argtypes = [l, l, d, d, P, i, i, P, P, P, l,
                                   P, P, P, P, P, P, P]
        L.orc_trace_uncached_2d.argtypes = [l, l, d, d, P, P, i, i, i, i, i,
                                            i, l, P, P]
        L.orc_raypath.argtypes = [P, l, l, l, P, l, P]
        L.orc_fibonacci.argtypes = [i, P]
        L.orc_build_cache_3d.argtypes = [P, l, i, u, i, i, P, P]
        L.orc_star_3d.argtypes = [i, d, d, d, i, P, P, P, P, P]
        L.orc_trace_3d.argtypes = [l, l, l, d, d, d, P, i, i, P, P, P, l, P, P, P, P, P]
        L.orc_build_cache_slow_2d.argtypes = [P, l, i, u, i, P, P]
        L.orc_trace_cells_2d.argtypes = [l, l, i, d, d, P, l, i, i, P, P, P, P, P, l, i,
                                         P, P, P, P, P]
        L.orc_trace_mspm_2d.argtypes = [l, l, i, d, d, P, P, l, i, i, i, l, i,
                                        P, P, P, P, P, P]
        L.orc_trace_blocks_3d.argtypes = [l, l, l, i, d, d, d, P, l, i, P, P, P, l, i,
                                          P, P, P, P, P]
        L.orc_slow_lookup.argtypes = [l, i, P, P, P, i, P, P, d, d, P]
        L.orc_trace_2d_slow.argtypes = [l, l, d, d, P, l, i, i, P, P, P, P, P, l, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ---------------------------------------------------------------- classes --

def class_from_thomsen(vp0, vs0, rho, eps, delta, gamma, tilt, azimuth, qp, qs):
    """13-double class: moduli (Thomsen 1986), Q per component (Qp on
    a11/a13/a33, Qs on a44/a66), rho, tilt, azimuth."""
    a5 = np.zeros(5)
    rc = lib().orc_thomsen(vp0, vs0, eps, delta, gamma, _p(a5))
    if rc != 0:
        raise ValueError("negative a13 radicand")
    return np.array([*a5, qp, qp, qp, qs, qs, rho, tilt, azimuth], dtype=np.float64)


def class_from_moduli(a11, a13, a33, a44, a66, q11, q13, q33, q44, q66,
                      rho=0.0, tilt=0.0, azimuth=0.0):
    return np.array([a11, a13, a33, a44, a66, q11, q13, q33, q44, q66,
                     rho, tilt, azimuth], dtype=np.float64)


# ------------------------------------------------------------ local solve --

def velocity(cls, mode, thR, thI, reading=MEV):
    """dict with complex v (2,), c, g (2,), p (2,) at (thR, thI), local frame."""
    out = np.zeros(14)
    c = np.ascontiguousarray(cls, dtype=np.float64)
    lib().orc_velocity(_p(c), mode, reading, thR, thI, _p(out))
    return {
        "v": np.array([out[0] + 1j * out[2], out[1] + 1j * out[3]]),
        "c": out[4] + 1j * out[5],
        "g": np.array([out[6] + 1j * out[7], out[8] + 1j * out[9]]),
        "p": np.array([out[10] + 1j * out[11], out[12] + 1j * out[13]]),
    }


def residual(cls, mode, thR, thI, reading=MEV):
    c = np.ascontiguousarray(cls, dtype=np.float64)
    return lib().orc_residual(_p(c), mode, reading, thR, thI)


def theta_imag(cls, mode, thR, reading=MEV):
    c = np.ascontiguousarray(cls, dtype=np.float64)
    out = np.zeros(1)
    rc = lib().orc_theta_imag(_p(c), mode, reading, thR, _p(out))
    return None if rc else float(out[0])


def solve(cls, mode, psi_local, reading=MEV, n_sweep=N_SWEEP):
    """One target local ray angle -> (dict of fields, status).  Direction in
    the local frame."""
    c = np.ascontiguousarray(cls, dtype=np.float64)
    out = np.zeros(NF)
    st = lib().orc_solve(_p(c), mode, reading, n_sweep, psi_local, _p(out))
    return dict(zip(FIELDS, out)), st


def sweep(cls, mode, reading=MEV, n_sweep=N_SWEEP):
    c = np.ascontiguousarray(cls, dtype=np.float64)
    thR, thI, psi = (np.zeros(n_sweep) for _ in range(3))
    ok = np.zeros(n_sweep, dtype=np.int32)
    lib().orc_sweep(_p(c), mode, reading, n_sweep, _p(thR), _p(thI), _p(psi), _p(ok))
    return thR, thI, psi, ok


def build_cache_2d(classes, n_dirs=360, mode_mask=0b111, reading=MEV,
                   n_sweep=N_SWEEP, subset=None):
    """Returns (fields [NF][3][K][n_cols], status [3][K][n_cols]); subset =
    ascending directions closed under reversal (None: all n_dirs)."""
    classes = np.ascontiguousarray(np.atleast_2d(classes), dtype=np.float64)
    K = classes.shape[0]
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int32)
    n_cols = n_dirs if sub is None else sub.size
    fields = np.full((NF, 3, K, n_cols), np.nan)
    status = np.zeros((3, K, n_cols), dtype=np.int32)
    rc = lib().orc_build_cache_2d_cols(_p(classes), K, n_dirs, _p(sub),
                                       0 if sub is None else sub.size, mode_mask,
                                       reading, n_sweep, _p(fields), _p(status))
    if rc:
        raise ValueError(f"orc_build_cache_2d failed rc={rc}")
    return fields, status


def star_subset(R, hx, hz, n_dirs=360):
    """Sorted unique bins of the forward star (closed under reversal)."""
    return np.unique(star_2d(R, hx, hz, n_dirs)[3]).astype(np.int32)


# ------------------------------------------------------------------ graph --

def star_2d(R, hx, hz, n_dirs=360):
    n = lib().orc_star_2d(R, hx, hz, n_dirs, None, None, None, None)
    ox = np.zeros(n, np.int32)
    oz = np.zeros(n, np.int32)
    L = np.zeros(n)
    b = np.zeros(n, np.int32)
    lib().orc_star_2d(R, hx, hz, n_dirs, _p(ox), _p(oz), _p(L), _p(b))
    return ox, oz, L, b


def trace_2d(nx, nz, hx, hz, class_id, R, V, A, status, src, n_dirs=360, subset=None,
             attenuation=True):
    """Dijkstra traveltimes for one mode from a cache slice V/A/status
    [K][n_cols].  class_id None: one class per node.  Returns dict of tauR,
    tauI, predP, predA, tstar, hopP, hopA; attenuation=False skips the
    attenuation field (tauI, predA, hopA come back None)."""
    n = nx * nz
    cid = None
    if class_id is not None:
        cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
        assert cid.size == n
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    st = np.ascontiguousarray(status, dtype=np.int32)
    out = {k: np.zeros(n) for k in ("tauR", "tauI", "tstar")}
    out.update({k: np.zeros(n, np.int32) for k in ("predP", "predA", "hopP", "hopA")})
    if not attenuation:
        out.update(tauI=None, predA=None, hopA=None)
    rc = lib().orc_trace_2d_cols(nx, nz, hx, hz, _p(cid), R, n_dirs, _p(sub),
                                 0 if sub is None else sub.size, _p(V), _p(A),
                                 _p(st), int(src), _p(out["tauR"]), _p(out["tauI"]),
                                 _p(out["predP"]), _p(out["predA"]), _p(out["tstar"]),
                                 _p(out["hopP"]), _p(out["hopA"]))
    if rc:
        raise ValueError(f"orc_trace_2d failed rc={rc}")
    return out


def trace_uncached_2d(nx, nz, hx, hz, class_id, classes, R, mode, field, src,
                      n_dirs=360, reading=MEV, n_sweep=N_SWEEP):
    n = nx * nz
    cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
    classes = np.ascontiguousarray(np.atleast_2d(classes), dtype=np.float64)
    tau = np.zeros(n)
    ns = ctypes.c_long(0)
    rc = lib().orc_trace_uncached_2d(nx, nz, hx, hz, _p(cid), _p(classes), R,
                                     n_dirs, mode, reading, n_sweep, field,
                                     int(src), _p(tau), ctypes.byref(ns))
    if rc:
        raise ValueError("orc_trace_uncached_2d failed")
    return tau, ns.value


def raypath(pred, src, rcv, capacity=None):
    """-> (rc, path array).  rc: 0 ok, 5 capacity, 6 unreachable, 7 cycle."""
    pred = np.ascontiguousarray(pred, dtype=np.int32)
    n = pred.size
    cap = n if capacity is None else capacity
    path = np.zeros(max(cap, 1), np.int64)
    ln = ctypes.c_long(0)
    rc = lib().orc_raypath(_p(pred), n, int(src), int(rcv), _p(path), cap,
                           ctypes.byref(ln))
    if rc == 5:
        return rc, ln.value
    return rc, (path[: ln.value].copy() if rc == 0 else None)


# --------------------------------------------------------------------- 3D --

N_FIB = 41253


def fibonacci(N=N_FIB):
    """Fibonacci ray directions [N, 3] (x, y, z), z down."""
    f = np.zeros((N, 3))
    lib().orc_fibonacci(N, _p(f))
    return f


def build_cache_3d(classes, N=N_FIB, mode_mask=0b011, reading=MEV, n_sweep=N_SWEEP):
    """(fields [NF][3][K][N], status [3][K][N]) on the Fibonacci directions,
    each entry the sagittal-plane solve at the polar angle to the axis."""
    classes = np.ascontiguousarray(np.atleast_2d(classes), dtype=np.float64)
    K = classes.shape[0]
    fields = np.full((NF, 3, K, N), np.nan)
    status = np.zeros((3, K, N), dtype=np.int32)
    rc = lib().orc_build_cache_3d(_p(classes), K, N, mode_mask, reading, n_sweep,
                                  _p(fields), _p(status))
    if rc:
        raise ValueError(f"orc_build_cache_3d failed rc={rc}")
    return fields, status


def star_3d(R, hx, hy, hz, N=N_FIB):
    n = lib().orc_star_3d(R, hx, hy, hz, N, None, None, None, None, None)
    ox, oy, oz, b = (np.zeros(n, np.int32) for _ in range(4))
    L = np.zeros(n)
    lib().orc_star_3d(R, hx, hy, hz, N, _p(ox), _p(oy), _p(oz), _p(L), _p(b))
    return ox, oy, oz, L, b


def trace_3d(nx, ny, nz, hx, hy, hz, class_id, R, V, A, status, src, N=N_FIB,
             outputs=("tauR", "tauI", "predP", "predA", "tstar")):
    """Dijkstra (tauR, tauI, predP, predA, tstar) on a 3D grid; node
    ix + nx (iy + ny iz); t* folds the attenuation weights along predP.
    Only the named outputs are computed (the others come back None)."""
    n = nx * ny * nz
    cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
    assert cid.size == n
    V = np.ascontiguousarray(V, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    st = np.ascontiguousarray(status, dtype=np.int32)
    out = {k: (np.zeros(n) if k in outputs else None) for k in ("tauR", "tauI", "tstar")}
    out.update({k: (np.zeros(n, np.int32) if k in outputs else None)
                for k in ("predP", "predA")})
    rc = lib().orc_trace_3d(nx, ny, nz, hx, hy, hz, _p(cid), R, N, _p(V), _p(A), _p(st),
                            int(src), _p(out["tauR"]), _p(out["tauI"]), _p(out["predP"]),
                            _p(out["predA"]), _p(out["tstar"]))
    if rc:
        raise ValueError(f"orc_trace_3d failed rc={rc}")
    return out


# ------------------------------------------------- slowness-sampled cache --

def build_cache_slow_2d(classes, n=360, mode_mask=0b111, reading=MEV):
    """The slowness-sampled cache: entry s of a class is the homogeneous
    solution at real slowness angle s 2 pi / n in the class's axis frame.
    Returns (fields [NF][3][K][n], status [3][K][n])."""
    classes = np.ascontiguousarray(np.atleast_2d(classes), dtype=np.float64)
    K = classes.shape[0]
    fields = np.full((NF, 3, K, n), np.nan)
    status = np.zeros((3, K, n), dtype=np.int32)
    rc = lib().orc_build_cache_slow_2d(_p(classes), K, n, mode_mask, reading, _p(fields),
                                       _p(status))
    if rc:
        raise ValueError(f"orc_build_cache_slow_2d failed rc={rc}")
    return fields, status


def slow_lookup(RX, RZ, status, R, hx, hz):
    """[K][|O|] sample of each class whose stored ray direction is closest
    to each star offset (-1 if none)."""
    RX = np.ascontiguousarray(RX, dtype=np.float64)
    RZ = np.ascontiguousarray(RZ, dtype=np.float64)
    st = np.ascontiguousarray(status, dtype=np.int32)
    K, n = RX.shape
    ox, oz, _, _ = star_2d(R, hx, hz, 4)
    best = np.zeros((K, ox.size), np.int32)
    lib().orc_slow_lookup(K, n, _p(RX), _p(RZ), _p(st), ox.size, _p(ox), _p(oz), hx, hz,
                          _p(best))
    return best


def trace_2d_slow(nx, nz, hx, hz, class_id, R, f_mode, st_mode, src):
    """Dijkstra on a slowness-sampled cache slice: f_mode = fields[:, mode]
    ([NF][K][n]), st_mode = status[mode].  Returns tauR, tauI, predP,
    predA, tstar."""
    n_nodes = nx * nz
    cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
    K, n = st_mode.shape
    V, A, RX, RZ = (np.ascontiguousarray(f_mode[i], dtype=np.float64) for i in (0, 1, 3, 4))
    st = np.ascontiguousarray(st_mode, dtype=np.int32)
    out = {k: np.zeros(n_nodes) for k in ("tauR", "tauI", "tstar")}
    out.update({k: np.zeros(n_nodes, np.int32) for k in ("predP", "predA")})
    rc = lib().orc_trace_2d_slow(nx, nz, hx, hz, _p(cid), K, R, n, _p(V), _p(A), _p(RX), _p(RZ),
                                 _p(st), int(src), _p(out["tauR"]), _p(out["tauI"]),
                                 _p(out["predP"]), _p(out["predA"]), _p(out["tstar"]))
    if rc:
        raise ValueError(f"orc_trace_2d_slow failed rc={rc}")
    return out


def cell_lattice(ncx, ncz, cn):
    """(NX, NZ, mask): lattice size of a cell network and which lattice
    points are nodes (on a cell edge)."""
    NX, NZ = ncx * cn + 1, ncz * cn + 1
    ix = np.arange(NX)[None, :]
    iz = np.arange(NZ)[:, None]
    return NX, NZ, ((ix % cn == 0) | (iz % cn == 0))


def trace_cells_2d(ncx, ncz, cn, hx, hz, class_id, f_mode, st_mode, src, sampling=0,
                   block=False):
    """Cell network (nodes on cell edges, all pairs within a cell; eqs 23-32):
    f_mode = fields[:, mode] ([NF][K][n_cols]), st_mode = status[mode];
    sampling 0 = ray-direction cache, 1 = slowness-sampled cache; block =
    the block marching instead of node Dijkstra.  Returns lattice-sized
    tauR, tauI, predP, predA, tstar."""
    NX, NZ, _ = cell_lattice(ncx, ncz, cn)
    n = NX * NZ
    cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
    assert cid.size == n
    K, nc = st_mode.shape
    V, A, RX, RZ = (np.ascontiguousarray(f_mode[i], dtype=np.float64) for i in (0, 1, 3, 4))
    st = np.ascontiguousarray(st_mode, dtype=np.int32)
    out = {k: np.zeros(n) for k in ("tauR", "tauI", "tstar")}
    out.update({k: np.zeros(n, np.int32) for k in ("predP", "predA")})
    rc = lib().orc_trace_cells_2d(ncx, ncz, cn, hx, hz, _p(cid), K, sampling, nc, _p(V), _p(A),
                                  _p(RX), _p(RZ), _p(st), int(src), int(bool(block)),
                                  _p(out["tauR"]), _p(out["tauI"]), _p(out["predP"]),
                                  _p(out["predA"]), _p(out["tstar"]))
    if rc:
        raise ValueError(f"orc_trace_cells_2d failed rc={rc}")
    return out


def block_lattice(ncx, ncy, ncz, cn):
    """(NX, NY, NZ, mask[NZ, NY, NX]): lattice of a 3D block network and which
    lattice points are nodes (on a block face)."""
    NX, NY, NZ = ncx * cn + 1, ncy * cn + 1, ncz * cn + 1
    ix = np.arange(NX)[None, None, :]
    iy = np.arange(NY)[None, :, None]
    iz = np.arange(NZ)[:, None, None]
    return NX, NY, NZ, ((ix % cn == 0) | (iy % cn == 0) | (iz % cn == 0))


def trace_blocks_3d(ncx, ncy, ncz, cn, hx, hy, hz, class_id, V, A, status, src, N=N_FIB,
                    block=False):
    """3D block network (nodes on block faces, all pairs within a block):
    V, A, status = one mode of a 3D cache ([K][N]); each segment reads the
    Fibonacci direction closest to it.  Returns lattice-sized tauR, tauI,
    predP, predA, tstar (node ix + NX (iy + NY iz))."""
    NX, NY, NZ, _ = block_lattice(ncx, ncy, ncz, cn)
    n = NX * NY * NZ
    cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
    assert cid.size == n
    V = np.ascontiguousarray(V, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    st = np.ascontiguousarray(status, dtype=np.int32)
    K = st.shape[0]
    assert V.shape == (K, N) and A.shape == (K, N) and st.shape == (K, N)
    out = {k: np.zeros(n) for k in ("tauR", "tauI", "tstar")}
    out.update({k: np.zeros(n, np.int32) for k in ("predP", "predA")})
    rc = lib().orc_trace_blocks_3d(ncx, ncy, ncz, cn, hx, hy, hz, _p(cid), K, N, _p(V), _p(A),
                                   _p(st), int(src), int(bool(block)), _p(out["tauR"]),
                                   _p(out["tauI"]), _p(out["predP"]), _p(out["predA"]),
                                   _p(out["tstar"]))
    if rc:
        raise ValueError(f"orc_trace_blocks_3d failed rc={rc}")
    return out


def trace_mspm_2d(ncx, ncz, cn, hx, hz, class_id, classes, mode, src, reading=MEV,
                  n_sweep=N_SWEEP, block=False):
    """MSPM (Algorithm 1) on the cell network: corner quantities from fresh
    solves at each segment's exact direction, non-corner nodes linearly
    reconstructed from the corners of their edge.  Returns lattice-sized
    tauR, tauI, predP, predA, tstar and n_solves (distinct solves)."""
    NX, NZ, _ = cell_lattice(ncx, ncz, cn)
    n = NX * NZ
    cid = np.ascontiguousarray(class_id, dtype=np.int32).reshape(-1)
    assert cid.size == n
    cls = np.ascontiguousarray(np.atleast_2d(classes), dtype=np.float64)
    out = {k: np.zeros(n) for k in ("tauR", "tauI", "tstar")}
    out.update({k: np.zeros(n, np.int32) for k in ("predP", "predA")})
    ns = ctypes.c_long(0)
    rc = lib().orc_trace_mspm_2d(ncx, ncz, cn, hx, hz, _p(cid), _p(cls), cls.shape[0], mode,
                                 reading, n_sweep, int(src), int(bool(block)), _p(out["tauR"]),
                                 _p(out["tauI"]), _p(out["predP"]), _p(out["predA"]),
                                 _p(out["tstar"]), ctypes.byref(ns))
    if rc:
        raise ValueError(f"orc_trace_mspm_2d failed rc={rc}")
    out["n_solves"] = ns.value
    return out
