"""Pins of the oracle's cell network (grid and nodal ray-network section,
eqs 23-24 and 27-32): nodes on cell edges, every pair of boundary nodes of a
cell joined by a segment, weights from the endpoint classes (eqs 28-30),
node Dijkstra and the paper's block marching from a heap of cells."""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_graph import py_bin, random_cache
from test_oracle_slow import random_slow_cache


def py_cell_edges(ncx, ncz, cn):
    """Every (i, j) pair of distinct boundary points of one cell, from the
    geometry: the lattice points of the closed cell rectangle that lie on
    its boundary."""
    NX = ncx * cn + 1
    edges = set()
    for cz in range(ncz):
        for cx in range(ncx):
            pts = []
            for z in range(cz * cn, (cz + 1) * cn + 1):
                for x in range(cx * cn, (cx + 1) * cn + 1):
                    if x in (cx * cn, (cx + 1) * cn) or z in (cz * cn, (cz + 1) * cn):
                        pts.append(x + NX * z)
            for a in pts:
                for b in pts:
                    if a != b:
                        edges.add((a, b))
    return sorted(edges)


def py_weights(edges, NX, hx, hz, cid, field, V, A, st, lookup):
    """eqs 28-30 per segment; lookup(k, dx, dz) -> column or -1."""
    out = []
    for i, j in edges:
        dx, dz = j % NX - i % NX, j // NX - i // NX
        ki, kj = cid[i], cid[j]
        ci, cj = lookup(ki, dx, dz), lookup(kj, dx, dz)
        L = math.sqrt((dx * hx) ** 2 + (dz * hz) ** 2)
        if ci < 0 or cj < 0 or st[ki, ci] or st[kj, cj]:
            w = math.inf
        elif field == 0:
            w = L / (0.5 * (V[ki, ci] + V[kj, cj]))
        else:
            w = L * (0.5 * (A[ki, ci] + A[kj, cj]))
        out.append((i, j, w))
    return out


def bellman_ford(n, wedges, src):
    tau = np.full(n, np.inf)
    tau[src] = 0.0
    changed = True
    while changed:
        changed = False
        for i, j, w in wedges:
            if tau[i] + w < tau[j]:
                tau[j] = tau[i] + w
                changed = True
    return tau


def ray_lookup(hx, hz, n_dirs):
    return lambda k, dx, dz: py_bin(dx, dz, hx, hz, n_dirs)


def slow_lookup_py(RX, RZ, st, hx, hz):
    def f(k, dx, dz):
        ex, ez = dx * hx, dz * hz
        ln = math.sqrt(ex * ex + ez * ez)
        ux, uz = ex / ln, ez / ln
        b, bd = -1, 0.0
        for q in range(RX.shape[1]):
            if st[k, q] & (O.ST_NO_BRACKET | O.ST_FLUID):
                continue
            d = RX[k, q] * ux + RZ[k, q] * uz
            if b < 0 or d > bd:
                b, bd = q, d
        return b
    return f


def fields_from(V, A, RX=None, RZ=None):
    K, n = V.shape
    f = np.full((O.NF, K, n), np.nan)
    f[0], f[1] = V, A
    if RX is not None:
        f[3], f[4] = RX, RZ
    return f


@pytest.mark.parametrize("ncx,ncz,cn,hx,hz", [(3, 2, 3, 10.0, 8.0), (2, 3, 2, 5.0, 5.0),
                                             (4, 1, 1, 7.0, 9.0)])
def test_ray_sampled_equals_bellman_ford(ncx, ncz, cn, hx, hz):
    """Dijkstra on the network equals Bellman-Ford over segments enumerated
    from the cell geometry, with bins and weights computed in Python,
    bitwise for both fields; and the block marching gives the same."""
    rng = np.random.default_rng(ncx * 10 + cn)
    K = 3
    V, A, st = random_cache(K, rng)
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = rng.integers(0, K, NX * NZ).astype(np.int32)
    src = int(np.flatnonzero(mask.reshape(-1))[3])
    edges = py_cell_edges(ncx, ncz, cn)
    f = fields_from(V, A)
    o = O.trace_cells_2d(ncx, ncz, cn, hx, hz, cid, f, st, src)
    ob = O.trace_cells_2d(ncx, ncz, cn, hx, hz, cid, f, st, src, block=True)
    for field, key in ((0, "tauR"), (1, "tauI")):
        we = py_weights(edges, NX, hx, hz, cid, field, V, A, st, ray_lookup(hx, hz, 360))
        ref = bellman_ford(NX * NZ, we, src)
        np.testing.assert_array_equal(o[key], ref)
        np.testing.assert_array_equal(ob[key], ref)


def test_slowness_sampled_equals_bellman_ford():
    """The same on a slowness-sampled cache with random stored ray
    directions: each end of a segment reads its class's closest stored
    direction."""
    rng = np.random.default_rng(21)
    K, n = 3, 60
    V, A, RX, RZ, st = random_slow_cache(K, n, rng)
    ncx, ncz, cn, hx, hz = 3, 3, 2, 10.0, 6.0
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = rng.integers(0, K, NX * NZ).astype(np.int32)
    src = 0
    edges = py_cell_edges(ncx, ncz, cn)
    f = fields_from(V, A, RX, RZ)
    o = O.trace_cells_2d(ncx, ncz, cn, hx, hz, cid, f, st, src, sampling=1)
    ob = O.trace_cells_2d(ncx, ncz, cn, hx, hz, cid, f, st, src, sampling=1, block=True)
    lk = slow_lookup_py(RX, RZ, st, hx, hz)
    for field, key in ((0, "tauR"), (1, "tauI")):
        ref = bellman_ford(NX * NZ, py_weights(edges, NX, hx, hz, cid, field, V, A, st, lk), src)
        np.testing.assert_array_equal(o[key], ref)
        np.testing.assert_array_equal(ob[key], ref)


def layered_cells(ncx, ncz, cn, K, seed):
    """Class per lattice point by depth band, K bands."""
    NX, NZ, _ = O.cell_lattice(ncx, ncz, cn)
    z = np.arange(NZ)
    band = np.minimum((z * K) // NZ, K - 1).astype(np.int32)
    return np.repeat(band[:, None], NX, 1)


@pytest.mark.parametrize("sampling", [0, 1])
def test_block_march_equals_dijkstra(sampling):
    """The block marching (heap of cells keyed by T_b, eq 24; all pairs of
    the taken cell relaxed until stable, eqs 31-32) reaches the same
    traveltimes as node Dijkstra bitwise on a layered TTI medium, so the
    predecessors and t* agree too."""
    cls = np.stack([O.class_from_thomsen(3000.0 + 400 * k, 1700.0 + 200 * k, 2300, 0.1 * k,
                                         0.05 * k, 0.08, math.radians(10 * k - 15), 0,
                                         60.0 + 20 * k, 40.0 + 10 * k) for k in range(3)])
    if sampling == 0:
        f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b011)
        fm, sm = f[:, 1], s[1]
    else:
        f, s = O.build_cache_slow_2d(cls, n=360, mode_mask=0b011)
        fm, sm = f[:, 1], s[1]
    ncx, ncz, cn = 9, 7, 4
    cid = layered_cells(ncx, ncz, cn, 3, 0)
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    src = 2 + NX * 0
    a = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, fm, sm, src, sampling=sampling)
    b = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, fm, sm, src, sampling=sampling,
                         block=True)
    for key in ("tauR", "tauI", "predP", "predA", "tstar"):
        np.testing.assert_array_equal(a[key], b[key])
    assert np.isfinite(a["tauR"][mask.reshape(-1)]).all()


def test_unit_cells_are_the_radius_one_star():
    """Cells of one interval: every lattice point is a node and each cell
    joins its 4 corners (4 sides, 2 diagonals), i.e. the 8 primitive offsets
    of radius 1, so the traveltimes equal the forward star's bitwise."""
    rng = np.random.default_rng(4)
    K = 4
    V, A, st = random_cache(K, rng)
    ncx, ncz, hx, hz = 13, 9, 10.0, 7.5
    NX, NZ, mask = O.cell_lattice(ncx, ncz, 1)
    assert mask.all()
    cid = rng.integers(0, K, NX * NZ).astype(np.int32)
    src = 5 + NX * 4
    c = O.trace_cells_2d(ncx, ncz, 1, hx, hz, cid, fields_from(V, A), st, src)
    s = O.trace_2d(NX, NZ, hx, hz, cid, 1, V, A, st, src)
    np.testing.assert_array_equal(c["tauR"], s["tauR"])
    np.testing.assert_array_equal(c["tauI"], s["tauI"])


def test_homogeneous_isotropic_straight_segments():
    """Isotropic elastic, one class: a node on the boundary of the source's
    cell is reached by the straight segment (tau = distance / V); every
    node's traveltime is at least its straight-line distance / V."""
    c = O.class_from_thomsen(3000.0, 1700.0, 2300, 0.0, 0.0, 0.0, 0.0, 0, np.inf, np.inf)
    f, s = O.build_cache_2d(c, n_dirs=360, mode_mask=0b001)
    ncx, ncz, cn, h = 6, 5, 5, 10.0
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = np.zeros(NX * NZ, np.int32)
    sx, sz = 10, 5  # corner shared by four cells
    src = sx + NX * sz
    o = O.trace_cells_2d(ncx, ncz, cn, h, h, cid, f[:, 0], s[0], src)
    X, Z = np.meshgrid(np.arange(NX), np.arange(NZ))
    dist = np.hypot((X - sx) * h, (Z - sz) * h).reshape(-1)
    node = mask.reshape(-1)
    assert np.all(o["tauR"][node] >= dist[node] / 3000.0 * (1 - 1e-14))
    near = node & (np.abs(X - sx) <= cn).reshape(-1) & (np.abs(Z - sz) <= cn).reshape(-1)
    np.testing.assert_allclose(o["tauR"][near], dist[near] / 3000.0, rtol=1e-15)
    assert np.all(o["tauI"][node] == 0.0)


def test_points_inside_cells_are_not_nodes():
    rng = np.random.default_rng(2)
    V, A, st = random_cache(2, rng)
    ncx, ncz, cn = 4, 3, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = rng.integers(0, 2, NX * NZ).astype(np.int32)
    o = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, fields_from(V, A), st, 0)
    inner = ~mask.reshape(-1)
    assert inner.sum() == ncx * ncz * (cn - 1) ** 2
    assert np.all(np.isinf(o["tauR"][inner])) and np.all(o["predP"][inner] == -1)
    assert np.all(np.isinf(o["tstar"][inner]))
    with pytest.raises(ValueError):  # a source inside a cell
        O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, fields_from(V, A), st,
                         int(np.flatnonzero(inner)[0]))


def test_predecessor_rule_and_tstar():
    """pred_j is the tight neighbour (sharing a cell) with the smallest
    (BFS hop over tight segments, node index); t* sums the attenuation
    weights along the propagation tree; checked in Python."""
    rng = np.random.default_rng(9)
    K = 2
    V, A, st = random_cache(K, rng, n_dirs=8)  # coarse bins: many equal weights
    ncx, ncz, cn, h = 4, 3, 3, 10.0
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = rng.integers(0, K, NX * NZ).astype(np.int32)
    src = 3
    o = O.trace_cells_2d(ncx, ncz, cn, h, h, cid, fields_from(V, A), st, src)
    edges = py_cell_edges(ncx, ncz, cn)
    lk = ray_lookup(h, h, 8)
    wR = {(i, j): w for i, j, w in py_weights(edges, NX, h, h, cid, 0, V, A, st, lk)}
    wI = {(i, j): w for i, j, w in py_weights(edges, NX, h, h, cid, 1, V, A, st, lk)}
    tau = o["tauR"]
    tight = {}
    for (i, j), w in wR.items():
        if np.isfinite(tau[j]) and tau[i] + w == tau[j]:
            tight.setdefault(j, []).append(i)
    hop = {src: 0}
    frontier = [src]
    while frontier:
        nxt = []
        for i in frontier:
            for (a, j), w in wR.items():
                if a == i and j not in hop and np.isfinite(tau[j]) and tau[i] + w == tau[j]:
                    hop[j] = hop[i] + 1
                    nxt.append(j)
        frontier = nxt
    n_ties = 0
    for j in np.flatnonzero(np.isfinite(tau)):
        if j == src:
            assert o["predP"][j] == -1
            continue
        cand = [i for i in tight[j] if i in hop]
        n_ties += len(cand) > 1
        assert o["predP"][j] == min(cand, key=lambda i: (hop[i], i))
        p = o["predP"][j]
        assert o["tstar"][j] == o["tstar"][p] + wI[(p, j)]
    assert n_ties > 0  # the rule was exercised
