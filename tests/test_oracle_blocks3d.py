"""Pins of the oracle's 3D block network (the 3D extension of the cell
network: nodes on block faces, every node pair of a block a straight
segment, eqs 27-31 with the Fibonacci cache of eq 35): unit blocks are the
radius-1 3D forward star, Bellman-Ford over segments listed and weighted in
Python from the block geometry, the block marching equal to node Dijkstra,
straight rays in a homogeneous isotropic medium, and the predecessor tree."""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_cells import bellman_ford

N_SMALL = 400


def tti_classes():
    return np.stack([
        O.class_from_thomsen(3000.0, 1700.0, 2300, 0.15, 0.05, 0.1, math.radians(25), 0.4,
                             50.0, 30.0),
        O.class_from_thomsen(3600.0, 2000.0, 2400, 0.05, 0.0, 0.05, math.radians(-10), 1.9,
                             80.0, 60.0),
        O.class_from_thomsen(2500.0, 1300.0, 2100, 0.25, 0.1, 0.2, math.radians(40), -0.7,
                             30.0, 20.0)])


@pytest.fixture(scope="module")
def cache():
    f, s = O.build_cache_3d(tti_classes(), N=N_SMALL, mode_mask=0b011)
    return f, s


def py_block_edges(ncx, ncy, ncz, cn):
    """Every (i, j) pair of distinct face points of one block, from the
    geometry: the lattice points of the closed box with a coordinate on
    one of its faces."""
    NX, NY = ncx * cn + 1, ncy * cn + 1
    edges = set()
    for bz in range(ncz):
        for by in range(ncy):
            for bx in range(ncx):
                lo = (bx * cn, by * cn, bz * cn)
                pts = []
                for z in range(lo[2], lo[2] + cn + 1):
                    for y in range(lo[1], lo[1] + cn + 1):
                        for x in range(lo[0], lo[0] + cn + 1):
                            if (x in (lo[0], lo[0] + cn) or y in (lo[1], lo[1] + cn)
                                    or z in (lo[2], lo[2] + cn)):
                                pts.append(x + NX * (y + NY * z))
                for a in pts:
                    for b in pts:
                        if a != b:
                            edges.add((a, b))
    return sorted(edges)


def py_fib_column(F, dx, dy, dz, hx, hy, hz):
    """Closest Fibonacci direction to the segment: the largest dot product
    with its unit vector, the first index among equals."""
    ex, ey, ez = dx * hx, dy * hy, dz * hz
    ln = math.sqrt(ex * ex + ez * ez + ey * ey)
    u = (ex / ln, ey / ln, ez / ln)
    d = F[:, 0] * u[0] + F[:, 1] * u[1] + F[:, 2] * u[2]
    return int(np.argmax(d)), ln


def py_block_weights(edges, NX, NY, h, cid, field, V, A, st, F):
    out = []
    memo = {}
    for i, j in edges:
        xi, yi, zi = i % NX, (i // NX) % NY, i // (NX * NY)
        xj, yj, zj = j % NX, (j // NX) % NY, j // (NX * NY)
        key = (xj - xi, yj - yi, zj - zi)
        if key not in memo:
            memo[key] = py_fib_column(F, *key, *h)
        c, L = memo[key]
        ki, kj = cid[i], cid[j]
        if st[ki, c] or st[kj, c]:
            w = math.inf
        elif field == 0:
            w = L / (0.5 * (V[ki, c] + V[kj, c]))
        else:
            w = L * (0.5 * (A[ki, c] + A[kj, c]))
        out.append((i, j, w))
    return out


def random_map(shape, K, seed):
    return np.random.default_rng(seed).integers(0, K, int(np.prod(shape))).astype(np.int32)


def test_block_lattice_counts():
    """Face points of the lattice: all points minus the block interiors."""
    for (ncx, ncy, ncz, cn) in ((2, 3, 2, 3), (1, 1, 1, 4), (3, 2, 1, 1)):
        NX, NY, NZ, mask = O.block_lattice(ncx, ncy, ncz, cn)
        assert mask.sum() == NX * NY * NZ - ncx * ncy * ncz * (cn - 1) ** 3
        assert len(py_block_edges(1, 1, 1, cn)) == ((cn + 1) ** 3 - (cn - 1) ** 3) * (
            (cn + 1) ** 3 - (cn - 1) ** 3 - 1)


@pytest.mark.parametrize("mode", [O.QP, O.QSV])
def test_unit_blocks_are_the_radius_1_star(cache, mode):
    """cn = 1: every lattice point is a node and a block's pairs are the 26
    neighbour offsets, the radius-1 3D forward star with the same closest-
    direction rule; traveltimes equal the 3D star oracle's bitwise."""
    f, s = cache
    ncx, ncy, ncz = 5, 4, 6
    h = (10.0, 12.5, 8.0)
    cid = random_map((ncz + 1, ncy + 1, ncx + 1), 3, 11)
    for src in (0, 37):
        b = O.trace_blocks_3d(ncx, ncy, ncz, 1, *h, cid, f[0, mode], f[1, mode], s[mode], src,
                              N=N_SMALL)
        r = O.trace_3d(ncx + 1, ncy + 1, ncz + 1, *h, cid, 1, f[0, mode], f[1, mode], s[mode],
                       src, N=N_SMALL)
        np.testing.assert_array_equal(b["tauR"], r["tauR"])
        np.testing.assert_array_equal(b["tauI"], r["tauI"])


@pytest.mark.parametrize("cn,h", [(2, (10.0, 10.0, 10.0)), (3, (8.0, 11.0, 9.5))])
def test_equals_bellman_ford_with_python_edges(cache, cn, h):
    """Traveltimes equal Bellman-Ford over the block pairs listed and
    weighted in Python (eqs 28-30, closest Fibonacci direction), bitwise,
    for both fields; a node inside a block stays unreached."""
    f, s = cache
    ncx, ncy, ncz = 2, 2, 2
    NX, NY, NZ, mask = O.block_lattice(ncx, ncy, ncz, cn)
    cid = random_map((NZ, NY, NX), 3, cn)
    F = O.fibonacci(N_SMALL)
    edges = py_block_edges(ncx, ncy, ncz, cn)
    src = 1 + NX * (0 + NY * cn)          # on the face z = cn, off the corners
    o = O.trace_blocks_3d(ncx, ncy, ncz, cn, *h, cid, f[0, 0], f[1, 0], s[0], src, N=N_SMALL)
    for field, key in ((0, "tauR"), (1, "tauI")):
        we = py_block_weights(edges, NX, NY, h, cid, field, f[0, 0], f[1, 0], s[0], F)
        np.testing.assert_array_equal(o[key], bellman_ford(NX * NY * NZ, we, src))
    m = mask.reshape(-1)
    assert np.isfinite(o["tauR"][m]).all() and np.isinf(o["tauR"][~m]).all()
    assert np.all(o["predP"][~m] == -1)


def test_block_march_equals_dijkstra(cache):
    f, s = cache
    ncx, ncy, ncz, cn = 3, 2, 3, 3
    NX, NY, NZ, _ = O.block_lattice(ncx, ncy, ncz, cn)
    cid = (np.arange(NZ)[:, None, None] * 3 // NZ).repeat(NY, 1).repeat(NX, 2).astype(np.int32)
    for mode in (O.QP, O.QSV):
        a = O.trace_blocks_3d(ncx, ncy, ncz, cn, 10, 10, 10, cid, f[0, mode], f[1, mode],
                              s[mode], 5, N=N_SMALL)
        b = O.trace_blocks_3d(ncx, ncy, ncz, cn, 10, 10, 10, cid, f[0, mode], f[1, mode],
                              s[mode], 5, N=N_SMALL, block=True)
        for key in ("tauR", "tauI", "predP", "predA", "tstar"):
            np.testing.assert_array_equal(a[key], b[key])


def test_isotropic_straight_rays():
    """Homogeneous isotropic elastic medium: a node sharing a block with the
    source is reached along the straight segment, tau = |d| / Vp; every
    other node is no earlier than that (the triangle inequality); tau_I and
    t* are 0."""
    c = O.class_from_thomsen(3000.0, 1700.0, 2300, 0.0, 0.0, 0.0, 0.0, 0.0, np.inf, np.inf)
    f, s = O.build_cache_3d(c, N=N_SMALL, mode_mask=0b001)
    ncx, ncy, ncz, cn = 3, 3, 2, 3
    h = (10.0, 7.0, 12.0)
    NX, NY, NZ, mask = O.block_lattice(ncx, ncy, ncz, cn)
    cid = np.zeros(NX * NY * NZ, np.int32)
    sx, sy, sz = 3, 4, 0
    src = sx + NX * (sy + NY * sz)
    o = O.trace_blocks_3d(ncx, ncy, ncz, cn, *h, cid, f[0, 0], f[1, 0], s[0], src, N=N_SMALL)
    z, y, x = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    d = np.sqrt(((x - sx) * h[0]) ** 2 + ((y - sy) * h[1]) ** 2 + ((z - sz) * h[2]) ** 2)
    d = d.reshape(-1)
    t = o["tauR"]
    m = mask.reshape(-1)
    shared = m & (x.reshape(-1) >= 3) & (x.reshape(-1) <= 6) & (y.reshape(-1) >= 3) & (
        y.reshape(-1) <= 6) & (z.reshape(-1) <= 3)
    np.testing.assert_allclose(t[shared], d[shared] / 3000.0, rtol=1e-12)
    assert np.all(t[m] >= d[m] / 3000.0 * (1 - 1e-12))
    assert np.all(o["tauI"][m] == 0.0) and np.all(o["tstar"][m] == 0.0)


def test_pred_tree_is_tight_and_folds_tstar(cache):
    """Each predecessor shares a block with its node and the segment is tight
    (tau_p + w = tau_j); among tight neighbours it has the fewest hops, then
    the lowest index; t* is the attenuation folded along the tree."""
    f, s = cache
    ncx, ncy, ncz, cn = 2, 2, 2, 2
    h = (9.0, 10.0, 11.0)
    NX, NY, NZ, mask = O.block_lattice(ncx, ncy, ncz, cn)
    cid = random_map((NZ, NY, NX), 3, 5)
    F = O.fibonacci(N_SMALL)
    src = 12
    o = O.trace_blocks_3d(ncx, ncy, ncz, cn, *h, cid, f[0, 0], f[1, 0], s[0], src, N=N_SMALL)
    edges = py_block_edges(ncx, ncy, ncz, cn)
    w0 = {(i, j): w for i, j, w in py_block_weights(edges, NX, NY, h, cid, 0, f[0, 0], f[1, 0],
                                                    s[0], F)}
    w1 = {(i, j): w for i, j, w in py_block_weights(edges, NX, NY, h, cid, 1, f[0, 0], f[1, 0],
                                                    s[0], F)}
    t, p = o["tauR"], o["predP"]
    tight = {}
    for (i, j), w in w0.items():
        if np.isfinite(t[j]) and t[i] + w == t[j]:
            tight.setdefault(j, []).append(i)
    # hops: BFS over tight segments from the source
    hop = {src: 0}
    frontier = [src]
    while frontier:
        nxt = []
        for i in frontier:
            for j, ins in tight.items():
                if j not in hop and i in ins:
                    hop[j] = hop[i] + 1
                    nxt.append(j)
        frontier = sorted(nxt)
    for j in range(NX * NY * NZ):
        if j == src or not mask.reshape(-1)[j]:
            assert p[j] == -1
            continue
        want = min(tight[j], key=lambda i: (hop.get(i, 1 << 30), i))
        assert p[j] == want
    ts = o["tstar"]
    for j in range(NX * NY * NZ):
        if p[j] >= 0:
            assert ts[j] == ts[p[j]] + w1[(p[j], j)]
