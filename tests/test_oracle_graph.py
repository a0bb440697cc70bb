"""Pins of the oracle's graph part (forward star, edge weights, Dijkstra,
predecessors, t*, raypaths) against brute force and closed forms.

The edge weight is restated here from the paper (eqs 27-30): an edge i -> j
with offset o has length L_o = |x_j - x_i| (eq 27), endpoint-averaged ray
velocity and attenuation at the bin of o (eq 28), propagation increment
L_o / Vbar (eq 29) and attenuation increment L_o * Abar (eq 30).  The two
fields are separate shortest-path problems (eqs 24, 31).
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O


def py_star(R, hx, hz, n_dirs=360):
    offs = []
    for oz in range(-R, R + 1):
        for ox in range(-R, R + 1):
            if (ox, oz) == (0, 0) or math.gcd(abs(ox), abs(oz)) != 1:
                continue
            offs.append((ox, oz))
    L = [math.sqrt((ox * hx) ** 2 + (oz * hz) ** 2) for ox, oz in offs]
    b = [py_bin(ox, oz, hx, hz, n_dirs) for ox, oz in offs]
    return offs, L, b


def py_bin(ox, oz, hx, hz, n_dirs):
    """Nearest of n_dirs equally spaced directions; on an exact tie the
    half-plane ox > 0 (or ox = 0, oz > 0) rounds up in angle and the other
    half-plane mirrors it, so bin(-o) = bin(o) + n_dirs/2."""
    if ox > 0 or (ox == 0 and oz > 0):
        x = math.degrees(math.atan2(ox * hx, oz * hz)) * n_dirs / 360.0
        return int(math.floor(x + 0.5)) % n_dirs
    return (py_bin(-ox, -oz, hx, hz, n_dirs) + n_dirs // 2) % n_dirs


def random_cache(K, rng, n_dirs=360, elastic=False):
    """Positive per-class V, A with the centrosymmetric copy."""
    h = n_dirs // 2
    V = rng.uniform(1500.0, 4500.0, (K, h))
    A = np.zeros((K, h)) if elastic else rng.uniform(1e-5, 1e-3, (K, h))
    return (np.concatenate([V, V], 1), np.concatenate([A, A], 1),
            np.zeros((K, n_dirs), np.int32))


def py_weight(field, V, A, ki, kj, L, b):
    if field == 0:
        return L / (0.5 * (V[ki, b] + V[kj, b]))
    return L * (0.5 * (A[ki, b] + A[kj, b]))


def py_edges(nx, nz, R, hx, hz, cid, V, A, field):
    offs, L, b = py_star(R, hx, hz)
    E = {}
    for iz in range(nz):
        for ix in range(nx):
            i = ix + nx * iz
            out = []
            for o, (ox, oz) in enumerate(offs):
                jx, jz = ix + ox, iz + oz
                if 0 <= jx < nx and 0 <= jz < nz:
                    j = jx + nx * jz
                    out.append((j, py_weight(field, V, A, cid[i], cid[j], L[o], b[o]), o))
            E[i] = out
    return E


# ----------------------------------------------------------------- star ---

def test_star_counts_and_bins():
    for R, n in zip(range(1, 6), [8, 16, 32, 48, 80]):
        ox, oz, L, b = O.star_2d(R, 10.0, 10.0)
        assert len(ox) == n
        offs, Lp, bp = py_star(R, 10.0, 10.0)
        assert list(zip(ox, oz)) == offs
        np.testing.assert_array_equal(L, Lp)
        np.testing.assert_array_equal(b, bp)
        assert len(set(b.tolist())) == n  # distinct 1-degree bins
        ang = np.degrees(np.arctan2(ox, oz))
        frac = np.abs((ang % 1.0) - 0.5)
        assert frac.min() > 0.06  # far from a rounding tie


@pytest.mark.parametrize("n_dirs", [360, 180, 90, 720, 36, 4])
@pytest.mark.parametrize("hx,hz", [(10.0, 10.0), (5.0, 7.5), (10.0, 5.0)])
def test_star_bins_nearest_and_antipodal(n_dirs, hx, hz):
    """bin(o) is a nearest tabulated direction of the edge vector (within
    half a step of its angle) and bin(-o) = bin(o) + n_dirs/2 for every
    step, including the 2-degree step where edges such as (1, 1) lie
    exactly half-way between two directions."""
    for R in range(1, 9):
        ox, oz, L, b = O.star_2d(R, hx, hz, n_dirs)
        offs, Lp, bp = py_star(R, hx, hz, n_dirs)
        np.testing.assert_array_equal(b, bp)
        step = 2 * np.pi / n_dirs
        ang = np.arctan2(ox * hx, oz * hz)
        miss = np.angle(np.exp(1j * (ang - b * step)))
        assert np.abs(miss).max() <= step / 2 * (1 + 1e-12)
        n = len(ox)
        # the star is ordered so that offset n-1-o is -o
        assert np.array_equal(ox[::-1], -ox) and np.array_equal(oz[::-1], -oz)
        np.testing.assert_array_equal(b[::-1], (b + n_dirs // 2) % n_dirs)
        sub = O.star_subset(R, hx, hz, n_dirs)
        assert set(((sub + n_dirs // 2) % n_dirs).tolist()) == set(sub.tolist())


# -------------------------------------------------------- brute force ---

@pytest.mark.parametrize("nx,nz", [(3, 3), (4, 2)])
def test_dijkstra_equals_exhaustive_simple_paths(nx, nz):
    """On tiny grids (R=1) tau_j is the minimum over ALL simple paths of the
    left-to-right FP64 fold of edge weights (eq 18 discretised) -- bitwise."""
    rng = np.random.default_rng(nx * 10 + nz)
    K = 3
    V, A, st = random_cache(K, rng)
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    for src in (0, nx * nz - 1, nx + 1 if nz > 1 else 1):
        r = O.trace_2d(nx, nz, 10.0, 10.0, cid, 1, V, A, st, src)
        for field, key in ((0, "tauR"), (1, "tauI")):
            E = py_edges(nx, nz, 1, 10.0, 10.0, cid, V, A, field)
            best = [math.inf] * (nx * nz)
            best[src] = 0.0

            def dfs(u, t, seen):
                for v, w, _ in E[u]:
                    if v in seen:
                        continue
                    tv = t + w
                    if tv < best[v]:
                        best[v] = tv
                    seen.add(v)
                    dfs(v, tv, seen)
                    seen.discard(v)

            dfs(src, 0.0, {src})
            assert np.array_equal(np.array(best), r[key])


def test_dijkstra_equals_bellman_ford_bitwise():
    """Label-correcting to the fixed point reaches the same FP64 values as
    Dijkstra, bitwise (any schedule: min over path folds)."""
    rng = np.random.default_rng(5)
    nx, nz, R, K = 9, 7, 3, 4
    V, A, st = random_cache(K, rng)
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    src = 3 + nx * 2
    r = O.trace_2d(nx, nz, 7.0, 5.0, cid, R, V, A, st, src)
    for field, key in ((0, "tauR"), (1, "tauI")):
        E = py_edges(nx, nz, R, 7.0, 5.0, cid, V, A, field)
        tau = [math.inf] * (nx * nz)
        tau[src] = 0.0
        for _ in range(nx * nz):
            changed = False
            for i in range(nx * nz):
                for j, w, _ in E[i]:
                    if tau[i] + w < tau[j]:
                        tau[j] = tau[i] + w
                        changed = True
            if not changed:
                break
        assert np.array_equal(np.array(tau), r[key])


# -------------------------------------------------------- closed forms ---

def farey_tau(X, Z, R):
    """Exact min over lattice paths with star steps of sum |o| (unit cost):
    decompose (X, Z) on the two star directions bracketing its angle."""
    offs, L, _ = py_star(R, 1.0, 1.0)
    ang = sorted((math.atan2(ox, oz), ox, oz) for ox, oz in offs)
    if (X, Z) == (0, 0):
        return 0.0
    t = math.atan2(X, Z)
    for k in range(len(ang)):
        a1, x1, z1 = ang[k]
        a2, x2, z2 = ang[(k + 1) % len(ang)]
        det = x1 * z2 - x2 * z1
        if det == 0:
            continue
        al = (X * z2 - x2 * Z) / det
        be = (x1 * Z - X * z1) / det
        if al >= -1e-12 and be >= -1e-12:
            assert abs(al - round(al)) < 1e-9 and abs(be - round(be)) < 1e-9
            return round(al) * math.hypot(x1, z1) + round(be) * math.hypot(x2, z2)
    raise AssertionError


@pytest.mark.parametrize("R", [1, 4, 5])
def test_homogeneous_isotropic_gauge_closed_form(R):
    """Homogeneous isotropic medium: graph traveltime = (a|u1| + b|u2|) h / V
    (unimodular decomposition on the bracketing star directions); straight
    rays along star directions give exactly r/V; tau_I = A * graph length."""
    nx = nz = 31
    h, Vv, Aa = 10.0, 3000.0, 2e-4
    V = np.full((1, 360), Vv)
    A = np.full((1, 360), Aa)
    st = np.zeros((1, 360), np.int32)
    cid = np.zeros(nx * nz, np.int32)
    src = 15 + nx * 15
    r = O.trace_2d(nx, nz, h, h, cid, R, V, A, st, src)
    for iz in range(nz):
        for ix in range(nx):
            g = farey_tau(ix - 15, iz - 15, R) * h
            j = ix + nx * iz
            assert abs(r["tauR"][j] - g / Vv) <= 1e-13 * max(g / Vv, 1e-30)
            assert abs(r["tauI"][j] - g * Aa) <= 1e-13 * max(g * Aa, 1e-30)
    # along the axis, exactly r / V
    for k in range(1, 15):
        assert abs(r["tauR"][15 + k + nx * 15] - k * h / Vv) < 1e-15


def test_central_symmetry_bitwise():
    """Homogeneous anisotropic class cache (centrosymmetric): tau(c+X) ==
    tau(c-X) bitwise for a centred source."""
    rng = np.random.default_rng(9)
    V, A, st = random_cache(1, rng)
    nx, nz = 41, 31
    cid = np.zeros(nx * nz, np.int32)
    c = 20 + nx * 15
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, 5, V, A, st, c)
    t = r["tauR"].reshape(nz, nx)
    assert np.array_equal(t, t[::-1, ::-1])
    t = r["tauI"].reshape(nz, nx)
    assert np.array_equal(t, t[::-1, ::-1])


def test_reciprocity():
    """Symmetric weights: tau_s(r) = tau_r(s) (to rounding of the fold)."""
    rng = np.random.default_rng(3)
    nx, nz, K = 25, 18, 5
    V, A, st = random_cache(K, rng)
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    pts = [0, 7 + nx * 3, 24 + nx * 17, 12 + nx * 9]
    fields = {s: O.trace_2d(nx, nz, 5.0, 5.0, cid, 4, V, A, st, s) for s in pts}
    for s, t in itertools.permutations(pts, 2):
        for key in ("tauR", "tauI"):
            a, b = fields[s][key][t], fields[t][key][s]
            assert abs(a - b) <= 1e-13 * a


def test_elastic_gives_zero_attenuation_fields():
    rng = np.random.default_rng(4)
    V, A, st = random_cache(3, rng, elastic=True)
    nx, nz = 20, 12
    cid = rng.integers(0, 3, nx * nz).astype(np.int32)
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, 3, V, A, st, 5)
    assert np.all(r["tauI"] == 0.0) and np.all(r["tstar"] == 0.0)
    # zero-weight edges: predecessors still form a BFS tree (hops = graph hops)
    assert np.all(r["predA"][np.arange(nx * nz) != 5] >= 0)


# ------------------------------------------------ predecessors, t*, paths ---

def _check_tree(nx, nz, R, hx, hz, cid, V, A, tau, pred, hop, src, field):
    offs, L, b = py_star(R, hx, hz)
    idx = {o: k for k, o in enumerate(offs)}
    n = nx * nz
    for j in range(n):
        if j == src:
            assert pred[j] == -1 and hop[j] == 0
            continue
        if not np.isfinite(tau[j]):
            assert pred[j] == -1
            continue
        # walk to the source; fold the weights from the source outwards
        path = [j]
        while path[-1] != src:
            p = pred[path[-1]]
            assert p >= 0 and len(path) <= n
            path.append(p)
        path = path[::-1]
        t = 0.0
        for a, c in zip(path[:-1], path[1:]):
            o = ((c % nx) - (a % nx), (c // nx) - (a // nx))
            k = idx[o]
            t = t + py_weight(field, V, A, cid[a], cid[c], L[k], b[k])
        assert t == tau[j]  # bitwise: the stored tree realises tau
        assert hop[j] == len(path) - 1


def test_predecessor_tree_realises_tau():
    rng = np.random.default_rng(21)
    nx, nz, R, K = 17, 13, 3, 3
    V, A, st = random_cache(K, rng)
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    src = 8
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, R, V, A, st, src)
    _check_tree(nx, nz, R, 5.0, 5.0, cid, V, A, r["tauR"], r["predP"], r["hopP"], src, 0)
    _check_tree(nx, nz, R, 5.0, 5.0, cid, V, A, r["tauI"], r["predA"], r["hopA"], src, 1)


def test_predecessor_rule_min_hop_then_offset():
    """pred_j is the tight neighbour with the smallest (hop, offset index)."""
    rng = np.random.default_rng(22)
    nx, nz, R = 15, 11, 2
    V = np.full((1, 360), 2000.0)  # homogeneous: many equal-time paths
    A = np.full((1, 360), 1e-4)
    st = np.zeros((1, 360), np.int32)
    cid = np.zeros(nx * nz, np.int32)
    src = 7 + nx * 5
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, R, V, A, st, src)
    offs, L, b = py_star(R, 5.0, 5.0)
    tau, hop, pred = r["tauR"], r["hopP"], r["predP"]
    for j in range(nx * nz):
        if j == src:
            continue
        jx, jz = j % nx, j // nx
        cands = []
        for k, (ox, oz) in enumerate(offs):
            ix, iz = jx - ox, jz - oz
            if 0 <= ix < nx and 0 <= iz < nz:
                i = ix + nx * iz
                w = py_weight(0, V, A, 0, 0, L[k], b[k])
                if tau[i] + w == tau[j]:
                    cands.append((hop[i], k, i))
        assert min(cands)[2] == pred[j]


def test_tstar_is_attenuation_along_propagation_tree():
    rng = np.random.default_rng(23)
    nx, nz, R, K = 14, 10, 2, 2
    V, A, st = random_cache(K, rng)
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    src = 3 + nx * 4
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, R, V, A, st, src)
    _check_tree(nx, nz, R, 5.0, 5.0, cid, V, A, r["tstar"], r["predP"], r["hopP"], src, 1)


def test_raypath_and_errors():
    rng = np.random.default_rng(24)
    V, A, st = random_cache(2, rng)
    nx, nz = 12, 9
    cid = rng.integers(0, 2, nx * nz).astype(np.int32)
    src, rcv = 2, 11 + nx * 8
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, 2, V, A, st, src)
    rc, path = O.raypath(r["predP"], src, rcv)
    assert rc == 0 and path[0] == src and path[-1] == rcv
    for a, c in zip(path[:-1], path[1:]):
        assert r["predP"][c] == a
    rc, need = O.raypath(r["predP"], src, rcv, capacity=2)
    assert rc == 5 and need == len(path)
    pred = r["predP"].copy()
    pred[rcv] = -1
    assert O.raypath(pred, src, rcv)[0] == 6
    pred = np.full(nx * nz, -1, np.int32)
    pred[5], pred[6] = 6, 5
    assert O.raypath(pred, src, 5)[0] == 7


def test_unusable_entries_block_edges():
    """An entry with no solution (or a fluid shear mode) makes its edges
    impassable: w = +inf."""
    rng = np.random.default_rng(25)
    V, A, st = random_cache(2, rng)
    st[1, :] = O.ST_FLUID
    nx, nz = 10, 10
    cid = np.zeros(nx * nz, np.int32)
    cid.reshape(nz, nx)[5:, :] = 1
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, 2, V, A, st, 0)
    t = r["tauR"].reshape(nz, nx)
    assert np.all(np.isfinite(t[:5])) and np.all(np.isinf(t[5:]))
    assert np.all(r["predP"].reshape(nz, nx)[5:] == -1)


@pytest.mark.slow
def test_cached_equals_uncached_bitwise():
    """The cache changes nothing but cost: Dijkstra with per-edge fresh solves
    at the binned direction (MSPM-style, no memo) gives bitwise the same
    traveltimes as the cached run (the paper reports < 1e-13 ms for qP)."""
    classes = np.stack([
        O.class_from_thomsen(3000.0, 1732.0, 2300, 0.2, 0.1, 0.15, np.radians(30), 0, 60, 40),
        O.class_from_thomsen(3600.0, 2000.0, 2400, 0.1, -0.05, 0.1, np.radians(-10), 0, 90, 54),
    ])
    nx, nz, R, ns = 5, 4, 2, 96
    cid = np.array([0] * 10 + [1] * 10, np.int32)
    f, st = O.build_cache_2d(classes, mode_mask=0b011, n_sweep=ns)
    for mode in (O.QP, O.QSV):
        r = O.trace_2d(nx, nz, 10.0, 10.0, cid, R, f[0, mode], f[1, mode], st[mode], 2)
        for field, key in ((0, "tauR"), (1, "tauI")):
            tau, nsolve = O.trace_uncached_2d(nx, nz, 10.0, 10.0, cid, classes, R,
                                              mode, field, 2, n_sweep=ns)
            assert nsolve > 0
            assert np.array_equal(tau, r[key])


def test_zero_weight_ties_use_min_hop_then_offset():
    """Elastic attenuation field: every edge weighs 0, so every neighbour is
    tight.  The predecessor must still be the min-(hop, offset index) one,
    which keeps the tree acyclic with hops equal to graph (BFS) hops."""
    rng = np.random.default_rng(26)
    V, A, st = random_cache(1, rng, elastic=True)
    nx, nz, R = 13, 9, 2
    cid = np.zeros(nx * nz, np.int32)
    src = 4 + nx * 3
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, R, V, A, st, src)
    offs, L, b = py_star(R, 5.0, 5.0)
    # BFS hops over the star graph, computed here independently
    hop = np.full(nx * nz, -1)
    hop[src] = 0
    frontier = [src]
    while frontier:
        nxt = []
        for i in frontier:
            for ox, oz in offs:
                jx, jz = i % nx + ox, i // nx + oz
                if 0 <= jx < nx and 0 <= jz < nz and hop[jx + nx * jz] < 0:
                    hop[jx + nx * jz] = hop[i] + 1
                    nxt.append(jx + nx * jz)
        frontier = nxt
    np.testing.assert_array_equal(r["hopA"], hop)
    for j in range(nx * nz):
        if j == src:
            continue
        jx, jz = j % nx, j // nx
        cands = [(hop[(jx - ox) + nx * (jz - oz)], k)
                 for k, (ox, oz) in enumerate(offs)
                 if 0 <= jx - ox < nx and 0 <= jz - oz < nz]
        h, k = min(cands)
        ox, oz = offs[k]
        assert r["predA"][j] == (jx - ox) + nx * (jz - oz)
    _check_tree(nx, nz, R, 5.0, 5.0, cid, V, A, r["tauI"], r["predA"], r["hopA"], src, 1)


def test_subset_cache_equals_full_cache_columns(rock_table):
    """A cache restricted to the star's directions stores exactly the full
    cache's values in those columns (same solve, different storage)."""
    r = rock_table[0]
    cls = np.stack([O.class_from_moduli(*(r[:5] * 1e6), *r[5:10], tilt=0.3),
                    O.class_from_thomsen(3000.0, 1732.0, 2300, 0.2, 0.1, 0.15, -0.2, 0, 60, 40)])
    sub = O.star_subset(3, 10.0, 10.0)
    f, s = O.build_cache_2d(cls, mode_mask=0b011, n_sweep=360)
    fs, ss = O.build_cache_2d(cls, mode_mask=0b011, n_sweep=360, subset=sub)
    for m in (0, 1):
        assert np.array_equal(fs[:, m], f[:, m][:, :, sub], equal_nan=True)
        assert np.array_equal(ss[m], s[m][:, sub])


def test_per_node_trace_equals_class_trace():
    """One class per node (no class map) with the star subset gives bitwise
    the traveltimes of the class-map form."""
    rng = np.random.default_rng(31)
    nx, nz, R, K = 14, 9, 3, 3
    V, A, st = random_cache(K, rng)
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    sub = O.star_subset(R, 5.0, 5.0)
    Vn, An, sn = V[cid][:, sub], A[cid][:, sub], st[cid][:, sub]
    a = O.trace_2d(nx, nz, 5.0, 5.0, cid, R, V, A, st, 17)
    b = O.trace_2d(nx, nz, 5.0, 5.0, None, R, Vn, An, sn, 17, subset=sub)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
