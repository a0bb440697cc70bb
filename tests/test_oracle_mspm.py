"""Pins of the oracle's MSPM form (Algorithm 1 on the cell network): corner
quantities from fresh solves at each segment's exact direction, nodes
between corners reconstructed linearly from the two corners of their edge,
then the cell network's shortest paths (eqs 28-31)."""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_cells import bellman_ford


def wrap_pi(a):
    while a > math.pi:
        a -= 2.0 * math.pi
    while a <= -math.pi:
        a += 2.0 * math.pi
    return a


BAD = O.ST_NO_BRACKET | O.ST_FLUID | O.ST_NONPHYS | O.ST_NOCONV


def py_corner(cls_row, mode, psi, memo, key, n_sweep):
    """Fresh solve at global ray angle psi with the cache entries' status
    rules, through the oracle's single-direction solve."""
    if key not in memo:
        f, st = O.solve(cls_row, mode, wrap_pi(psi - cls_row[11]), n_sweep=n_sweep)
        if not st & O.ST_NO_BRACKET:
            if not (f["A"] >= 0.0) or not np.isfinite(f["V"]) or not (f["V"] > 0.0):
                st |= O.ST_NONPHYS
            if not (f["res"] <= 1e-9):
                st |= O.ST_NOCONV
        memo[key] = (f["V"], f["A"], st)
    return memo[key]


def py_mspm_weights(ncx, ncz, cn, hx, hz, cid, classes, mode, field, n_sweep):
    """(i, j, w) for every segment of every cell, the reconstruction written
    from the cell geometry."""
    NX = ncx * cn + 1
    memo = {}
    out = []
    for cz in range(ncz):
        for cx in range(ncx):
            x0, z0 = cx * cn, cz * cn
            pts = [(x, z) for z in range(z0, z0 + cn + 1) for x in range(x0, x0 + cn + 1)
                   if x in (x0, x0 + cn) or z in (z0, z0 + cn)]
            for (ax, az) in pts:
                for (bx, bz) in pts:
                    if (ax, az) == (bx, bz):
                        continue
                    dx, dz = bx - ax, bz - az
                    cdx, cdz = (dx, dz) if (dx > 0 or (dx == 0 and dz > 0)) else (-dx, -dz)
                    psi = math.atan2(cdx * hx, cdz * hz)

                    def q(x, z):
                        def corner(px, pz):
                            k = cid[px + NX * pz]
                            return py_corner(classes[k], mode, psi, memo, (k, cdx, cdz),
                                             n_sweep)
                        if x in (x0, x0 + cn) and z in (z0, z0 + cn):
                            return corner(x, z)
                        if z in (z0, z0 + cn):
                            c1, c2, t = corner(x0, z), corner(x0 + cn, z), (x - x0) / cn
                        else:
                            c1, c2, t = corner(x, z0), corner(x, z0 + cn), (z - z0) / cn
                        return (c1[0] + t * (c2[0] - c1[0]), c1[1] + t * (c2[1] - c1[1]),
                                c1[2] | c2[2])

                    Va, Aa, sa = q(ax, az)
                    Vb, Ab, sb = q(bx, bz)
                    L = math.sqrt((dx * hx) ** 2 + (dz * hz) ** 2)
                    if (sa | sb) & BAD:
                        w = math.inf
                    elif field == 0:
                        w = L / (0.5 * (Va + Vb))
                    else:
                        w = L * (0.5 * (Aa + Ab))
                    out.append((ax + NX * az, bx + NX * bz, w))
    return out


def two_classes():
    return np.stack([O.class_from_thomsen(3000.0, 1700.0, 2300, 0.15, 0.05, 0.1,
                                          math.radians(20), 0, 50.0, 30.0),
                     O.class_from_thomsen(3600.0, 2000.0, 2400, 0.05, 0.0, 0.05,
                                          math.radians(-10), 0, 80.0, 60.0)])


@pytest.mark.parametrize("mode", [O.QP, O.QSV])
def test_mspm_equals_bellman_ford_with_python_reconstruction(mode):
    """Traveltimes equal Bellman-Ford over segments whose weights come from
    the oracle's single-direction solve at each segment's exact angle and a
    reconstruction written in Python from the cell geometry, bitwise."""
    cls = two_classes()
    ncx, ncz, cn, hx, hz = 3, 2, 3, 10.0, 8.0
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    rng = np.random.default_rng(3)
    cid = rng.integers(0, 2, NX * NZ).astype(np.int32)
    src = 3
    o = O.trace_mspm_2d(ncx, ncz, cn, hx, hz, cid, cls, mode, src, n_sweep=720)
    for field, key in ((0, "tauR"), (1, "tauI")):
        we = py_mspm_weights(ncx, ncz, cn, hx, hz, cid, cls, mode, field, 720)
        np.testing.assert_array_equal(o[key], bellman_ford(NX * NZ, we, src))


def test_block_march_equals_dijkstra():
    cls = two_classes()
    ncx, ncz, cn = 6, 4, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = (np.arange(NZ)[:, None] * 2 // NZ).repeat(NX, 1).astype(np.int32)
    a = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 10.0, cid, cls, O.QSV, 2, n_sweep=720)
    b = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 10.0, cid, cls, O.QSV, 2, n_sweep=720, block=True)
    for key in ("tauR", "tauI", "predP", "predA", "tstar"):
        np.testing.assert_array_equal(a[key], b[key])


def test_isotropic_equals_cached_cells():
    """Isotropic elastic, one class: every solve gives V = Vp (to rounding),
    the reconstruction between equal corners is exact, so MSPM's traveltimes
    equal the cached cell network's; tau_I is 0."""
    c = O.class_from_thomsen(3000.0, 1700.0, 2300, 0.0, 0.0, 0.0, 0.0, 0, np.inf, np.inf)
    ncx, ncz, cn = 5, 4, 5
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = np.zeros(NX * NZ, np.int32)
    m = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 10.0, cid, c[None], O.QP, 7, n_sweep=720)
    f, s = O.build_cache_2d(c, n_dirs=360, mode_mask=0b001, n_sweep=720)
    h = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, f[:, 0], s[0], 7)
    node = mask.reshape(-1)
    np.testing.assert_allclose(m["tauR"][node], h["tauR"][node], rtol=1e-13)
    assert np.all(m["tauI"][node] == 0.0)
    # one solve per canonical direction of the cell's segments
    assert m["n_solves"] == ((2 * cn + 1) ** 2 - 1) // 2


def test_uniform_medium_close_to_fine_cache():
    """One VTI class: corners all alike, so MSPM is the cell network read at
    exact directions; a 0.1-degree cache comes within its binning error."""
    c = two_classes()[:1]
    ncx, ncz, cn = 6, 5, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = np.zeros(NX * NZ, np.int32)
    m = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 10.0, cid, c, O.QP, 0, n_sweep=1440)
    f, s = O.build_cache_2d(c, n_dirs=3600, mode_mask=0b001)
    h = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, f[:, 0], s[0], 0)
    node = mask.reshape(-1)
    rel = np.abs(m["tauR"][node] - h["tauR"][node]) / np.maximum(h["tauR"][node], 1e-300)
    assert rel.max() < 2e-4 and rel.max() > 0.0


def test_reconstruction_reads_only_corners():
    """A node between two corners ignores its own class: changing the class
    of the non-corner nodes alone leaves MSPM's field unchanged, while the
    cached cell network (which reads every node's class) changes."""
    cls = two_classes()
    ncx, ncz, cn = 5, 4, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    X, Z = np.meshgrid(np.arange(NX), np.arange(NZ))
    corner = ((X % cn == 0) & (Z % cn == 0)).reshape(-1)
    cid0 = (Z >= 8).astype(np.int32).reshape(-1)
    cid1 = cid0.copy()
    cid1[~corner] = 1 - cid1[~corner]
    a = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 10.0, cid0, cls, O.QP, 0, n_sweep=720)
    b = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 10.0, cid1, cls, O.QP, 0, n_sweep=720)
    for key in ("tauR", "tauI", "predP", "tstar"):
        np.testing.assert_array_equal(a[key], b[key])
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b001, n_sweep=720)
    c0 = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid0, f[:, 0], s[0], 0)
    c1 = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid1, f[:, 0], s[0], 0)
    assert not np.array_equal(c0["tauR"], c1["tauR"])
    assert np.isfinite(a["tauR"][mask.reshape(-1)]).all()
    assert np.all(a["predP"][~mask.reshape(-1)] == -1)
