"""The tree relaxation's fixed point (host-side emulation, no GPU).

The GPU computes predecessors and t* by a label-correcting relaxation over
the tight edges: key_j = min over tight in-edges i -> j of
(hop_i + 1, offset index), and t*_j = t*_p + w_I(p -> j) for the p its key
names, in whatever order its workgroups happen to run.  Here the same
update rule runs sequentially in random node orders until nothing changes;
every order must land on the oracle's predecessors, hop counts and t*
(eq 33 and the t* fold), bitwise.  The edge weights are rebuilt from the
oracle cache by eqs 28-30 and first checked to reproduce the oracle's
traveltimes bitwise.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _model_and_fields():
    m = W.small_layered(nx=16, nz=11, radius=2, seed=3)
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    f, s = O.build_cache_2d(cls, n_dirs=m.n_dirs, mode_mask=0b001, n_sweep=360)
    src = m.sources[0]
    o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, f[0, 0], f[1, 0], s[0], src)
    return m, f, s, src, o


def _weights(m, f, s):
    """w[field][(i, j, o)] by eqs 28-30, edge i -> j = i + o."""
    ox, oz, L, b = O.star_2d(m.radius, m.hx, m.hz, m.n_dirs)
    V, A, st = f[0, 0], f[1, 0], s[0]
    bad = O.ST_NO_BRACKET | O.ST_FLUID | O.ST_NONPHYS
    cid = np.asarray(m.class_id).reshape(-1)
    edges = []
    for j in range(m.nx * m.nz):
        jx, jz = j % m.nx, j // m.nx
        for k in range(len(ox)):
            ix, iz = jx - int(ox[k]), jz - int(oz[k])
            if not (0 <= ix < m.nx and 0 <= iz < m.nz):
                continue
            i = ix + m.nx * iz
            ki, kj, c = int(cid[i]), int(cid[j]), int(b[k])
            if (st[ki, c] & bad) or (st[kj, c] & bad):
                wr = wi = math.inf
            else:
                wr = float(L[k]) / (0.5 * (float(V[ki, c]) + float(V[kj, c])))
                wi = float(L[k]) * (0.5 * (float(A[ki, c]) + float(A[kj, c])))
            edges.append((i, j, k, wr, wi))
    return edges


def _relax_tree(n, src, tau, edges, field, fold, rng):
    """Random-order sweeps of the tree update until a sweep changes nothing."""
    ins = [[] for _ in range(n)]
    for (i, j, k, wr, wi) in edges:
        w = wr if field == 0 else wi
        if math.isfinite(tau[j]) and tau[i] + w == tau[j]:
            ins[j].append((i, k, wi))
    key = [None] * n
    key[src] = (0, 0)
    ts = [math.nan] * n
    ts[src] = 0.0
    for _ in range(10 * n):
        changed = False
        for j in rng.permutation(n):
            if j == src:
                continue
            best = key[j]
            for (i, k, _) in ins[j]:
                if key[i] is not None:
                    cand = (key[i][0] + 1, k)
                    if best is None or cand < best:
                        best = cand
            if best != key[j]:
                key[j] = best
                changed = True
            if fold and key[j] is not None:
                p, wi = next((i, wi) for (i, k, wi) in ins[j] if k == key[j][1])
                t = ts[p] + wi
                if not (t == ts[j] or (math.isnan(t) and math.isnan(ts[j]))):
                    ts[j] = t
                    changed = True
        if not changed:
            break
    else:
        raise AssertionError("tree relaxation did not settle")
    return key, ts


@pytest.fixture(scope="module")
def case():
    return _model_and_fields()


def test_rebuilt_weights_reproduce_oracle_traveltimes(case):
    """Bellman-Ford check: the rebuilt weights give the oracle's tau bitwise."""
    m, f, s, src, o = case
    edges = _weights(m, f, s)
    for field, name in ((0, "tauR"), (1, "tauI")):
        tau = np.asarray(o[name]).reshape(-1)
        best = np.full(tau.size, math.inf)
        best[src] = 0.0
        for (i, j, k, wr, wi) in edges:
            w = wr if field == 0 else wi
            best[j] = min(best[j], tau[i] + w)
        assert np.array_equal(best, tau), name


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tree_relaxation_any_order_gives_oracle_pred_hop_tstar(case, seed):
    m, f, s, src, o = case
    edges = _weights(m, f, s)
    n = m.nx * m.nz
    rng = np.random.default_rng(seed)
    ox, oz, _, _ = O.star_2d(m.radius, m.hx, m.hz, m.n_dirs)
    for field, tkey, pkey, hkey in ((0, "tauR", "predP", "hopP"), (1, "tauI", "predA", "hopA")):
        tau = [float(v) for v in np.asarray(o[tkey]).reshape(-1)]
        key, ts = _relax_tree(n, src, tau, edges, field, field == 0, rng)
        pred = np.full(n, -1, np.int64)
        hop = np.full(n, -1, np.int64)
        for j in range(n):
            if key[j] is None:
                continue
            hop[j] = key[j][0]
            if j != src:
                k = key[j][1]
                pred[j] = j - (int(ox[k]) + m.nx * int(oz[k]))
        assert np.array_equal(pred, np.asarray(o[pkey]).reshape(-1)), (seed, pkey)
        oh = np.asarray(o[hkey]).reshape(-1)
        reach = oh >= 0
        assert np.array_equal(hop[reach], oh[reach]), (seed, hkey)
        if field == 0:
            t = np.array([math.inf if math.isnan(v) else v for v in ts])
            assert np.array_equal(t, np.asarray(o["tstar"]).reshape(-1)), seed
