"""GPU parity of the cell network (nodes on cell edges, every boundary pair
of a cell a segment; eqs 23-24, 27-32): traveltimes, t* and predecessors
through the C ABI against the oracle's node Dijkstra, bitwise on imported
oracle caches (ray-direction and slowness-sampled, cell sides of 1 to 16
intervals, unordered and block-ordered rounds), the GPU's own cache traced
end to end, and the error paths."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from test_oracle_cells import layered_cells  # noqa: E402
from test_oracle_slow import random_slow_cache  # noqa: E402

KEYS = ("tauR", "tauI", "tstar", "predP", "predA")


def tree_levels(pred, src):
    """Levels of a predecessor tree (hop of its deepest node + 1)."""
    h = np.full(pred.size, -1, np.int64)
    h[src] = 0
    while True:
        m = (h < 0) & (pred >= 0)
        m[m] = h[pred[m]] >= 0
        if not m.any():
            return int(h.max()) + 1
        h[m] = h[pred[m]] + 1


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import chert_gpu
    return chert_gpu


def _C():
    import paper_2609_26108_amd as C
    return C


def tti_classes(K=3):
    return np.stack([O.class_from_thomsen(3000.0 + 400 * k, 1700.0 + 200 * k, 2300, 0.1 * k,
                                          0.05 * k, 0.08, np.radians(12 * k - 15), 0,
                                          60.0 + 20 * k, 40.0 + 10 * k) for k in range(K)])


def node_sources(ncx, ncz, cn, picks):
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    nodes = np.flatnonzero(mask.reshape(-1))
    return [int(nodes[int(p * (nodes.size - 1))]) for p in picks]


@pytest.mark.parametrize("cn,ncx,ncz,bucket", [(5, 12, 8, 0.0), (5, 12, 8, 8.0), (1, 30, 20, 0.0),
                                               (3, 15, 9, 4.0), (16, 4, 3, 0.0),
                                               (16, 4, 3, 64.0), (7, 6, 5, 1.0)])
def test_ray_cache_bitwise(G, cn, ncx, ncz, bucket):
    """Imported oracle ray-direction cache of three tilted TTI classes in
    depth bands; both modes, two sources; every output bitwise."""
    C = _C()
    cls = tti_classes()
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b011)
    desc = C.cache_desc(n_dirs=360, modes=(0, 1))
    cache = G.import_cache(f, s, desc, 3)
    cid = layered_cells(ncx, ncz, cn, 3, 0)
    srcs = node_sources(ncx, ncz, cn, (0.1, 0.77))
    h = 10.0 if cn < 8 else 4.0
    for mode in (0, 1):
        st = C.TraceStats()
        g = G.trace_cells(cache, desc, 3, ncx, ncz, cn, h, 0.8 * h, cid, mode, srcs,
                          bucket_width=bucket, stats=st)
        assert st.rounds[0] > 0 and st.tile_visits[0] > 0
        for si, src in enumerate(srcs):
            o = O.trace_cells_2d(ncx, ncz, cn, h, 0.8 * h, cid, f[:, mode], s[mode], src)
            for key in KEYS:
                assert np.array_equal(g[key][si], o[key]), (mode, si, key)
        # the reported BFS depth is the deepest predecessor tree of the call
        deepest = max(tree_levels(g[k][si], src) for si, src in enumerate(srcs)
                      for k in ("predP", "predA"))
        assert st.rounds[1] == deepest, (st.rounds[1], deepest)


@pytest.mark.parametrize("cn,bucket", [(4, 0.0), (6, 16.0)])
def test_slowness_cache_random_directions_bitwise(G, cn, bucket):
    """Stored ray directions at random angles (the per-end lookup picks
    different samples for the two end classes)."""
    C = _C()
    rng = np.random.default_rng(cn)
    K, n = 4, 90
    V, A, RX, RZ, st = random_slow_cache(K, n, rng)
    f = np.full((O.NF, 3, K, n), np.nan)
    s = np.zeros((3, K, n), np.int32)
    f[0, 0], f[1, 0], f[3, 0], f[4, 0] = V, A, RX, RZ
    s[0] = st
    ncx, ncz = 9, 7
    NX, NZ, _ = O.cell_lattice(ncx, ncz, cn)
    cid = rng.integers(0, K, NX * NZ).astype(np.int32)
    desc = C.cache_desc(n_dirs=n, modes=(0,), sampling=C.SAMPLE_SLOWNESS)
    cache = G.import_cache(f, s, desc, K)
    srcs = node_sources(ncx, ncz, cn, (0.0, 0.5))
    g = G.trace_cells(cache, desc, K, ncx, ncz, cn, 10.0, 6.0, cid, 0, srcs, bucket_width=bucket)
    for si, src in enumerate(srcs):
        o = O.trace_cells_2d(ncx, ncz, cn, 10.0, 6.0, cid, f[:, 0], s[0], src, sampling=1)
        for key in KEYS:
            assert np.array_equal(g[key][si], o[key]), (si, key)


def test_slowness_cache_of_classes_bitwise(G):
    """An oracle slowness-sampled cache of the TTI classes, both modes."""
    C = _C()
    cls = tti_classes()
    f, s = O.build_cache_slow_2d(cls, n=360, mode_mask=0b011)
    desc = C.cache_desc(n_dirs=360, modes=(0, 1), sampling=C.SAMPLE_SLOWNESS)
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncz, cn = 10, 8, 5
    cid = layered_cells(ncx, ncz, cn, 3, 0)
    srcs = node_sources(ncx, ncz, cn, (0.3,))
    for mode in (0, 1):
        g = G.trace_cells(cache, desc, 3, ncx, ncz, cn, 10.0, 10.0, cid, mode, srcs)
        o = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, f[:, mode], s[mode], srcs[0],
                             sampling=1)
        for key in KEYS:
            assert np.array_equal(g[key][0], o[key]), (mode, key)


def test_unit_cells_equal_radius_one_star(G):
    """Cells of one interval are the radius-1 forward star: the cell path's
    traveltimes equal the tile path's bitwise."""
    C = _C()
    cls = tti_classes()
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b001)
    desc = C.cache_desc(n_dirs=360, modes=(0,))
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncz = 40, 25
    cid = layered_cells(ncx, ncz, 1, 3, 0)
    src = 7 + 41 * 3
    a = G.trace_cells(cache, desc, 3, ncx, ncz, 1, 10.0, 10.0, cid, 0, [src])
    b = G.trace(cache, desc, 3, ncx + 1, ncz + 1, 10.0, 10.0, 1, cid, 0, [src])
    assert np.array_equal(a["tauR"], b["tauR"]) and np.array_equal(a["tauI"], b["tauI"])


def test_gpu_cache_end_to_end(G):
    """The GPU's own cache of the classes traced on the cell network against
    the oracle's cache and Dijkstra (1e-9)."""
    C = _C()
    cls = tti_classes()
    desc = C.cache_desc(n_dirs=360, modes=(1,), n_sweep=1440)
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    fo, so = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b010)
    ncx, ncz, cn = 20, 12, 5
    cid = layered_cells(ncx, ncz, cn, 3, 0)
    srcs = node_sources(ncx, ncz, cn, (0.05,))
    g = G.trace_cells(cache, desc, 3, ncx, ncz, cn, 10.0, 10.0, cid, 1, srcs, bucket_width=8.0)
    o = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, fo[:, 1], so[1], srcs[0])
    for key in ("tauR", "tauI", "tstar"):
        a, b = g[key][0], o[key]
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin)
        rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
        assert rel.max() <= 1e-9, (key, rel.max())


def test_errors_leave_outputs_untouched(G):
    C = _C()
    cls = tti_classes(2)
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b001)
    desc = C.cache_desc(n_dirs=360, modes=(0,))
    cache = G.import_cache(f, s, desc, 2)
    ncx, ncz, cn = 6, 4, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    n = NX * NZ
    cid = torch.zeros(n, dtype=torch.int32, device=G.DEV)
    cid[n // 2] = 7  # out of range
    g = C.make_cell_grid(ncx, ncz, cn, 10.0, 10.0, cid)
    o = C.trace_opts(C.OUT_TAU_R)
    out = torch.full((1, n), -5.0, dtype=torch.float64, device=G.DEV)
    ws = torch.empty(C.chert_trace_cells_workspace_bytes(desc, 2, g, 1, o), dtype=torch.uint8,
                     device=G.DEV)
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_cells(desc, cache, 2, g, 0, [0], o, out, workspace_dev=ws)
    assert e.value.code == C.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(out == -5.0)
    cid[n // 2] = 1
    inner = int(np.flatnonzero(~mask.reshape(-1))[0])
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_cells(desc, cache, 2, g, 0, [inner], o, out, workspace_dev=ws)
    assert e.value.code == C.ERR_INVALID_ARG
    with pytest.raises(C.ChertError) as e:  # round cap
        C.chert_trace_cells(desc, cache, 2, g, 0, [0], C.trace_opts(C.OUT_TAU_R, max_rounds=1),
                            out, workspace_dev=ws)
    assert e.value.code == C.ERR_NO_CONVERGENCE
    flag = torch.ones(1, dtype=torch.int32).pin_memory()
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_cells(desc, cache, 2, g, 0, [0],
                            C.trace_opts(C.OUT_TAU_R, abort_flag=flag), out, workspace_dev=ws)
    assert e.value.code == C.ERR_ABORTED
    C.chert_trace_cells(desc, cache, 2, g, 0, [0], o, out, workspace_dev=ws)
    torch.cuda.synchronize()
    t = out[0].cpu().numpy()
    assert t[0] == 0.0 and np.isfinite(t[mask.reshape(-1)]).all()
    assert np.isinf(t[~mask.reshape(-1)]).all()


@pytest.mark.parametrize("bucket", [0.0, 16.0])
def test_full_size_layered_network_bitwise(G, bucket):
    """The benchmark's network: 80x40 cells of 5x5 intervals on the 5-layer
    401x201 lattice at 5 m, qSV through an imported oracle cache, every
    output bitwise against the oracle."""
    import workloads as W
    C = _C()
    m = W.config2()
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b010)
    desc = C.cache_desc(n_dirs=360, modes=(1,))
    K = cls.shape[0]
    cache = G.import_cache(f, s, desc, K)
    cn = 5
    ncx, ncz = (m.nx - 1) // cn, (m.nz - 1) // cn
    g = G.trace_cells(cache, desc, K, ncx, ncz, cn, m.hx, m.hz, m.class_id, 1, m.sources,
                      bucket_width=bucket)
    o = O.trace_cells_2d(ncx, ncz, cn, m.hx, m.hz, m.class_id, f[:, 1], s[1], m.sources[0])
    for key in KEYS:
        assert np.array_equal(g[key][0], o[key]), key


@pytest.mark.parametrize("cn,ncx,ncz", [(1, 1, 1), (16, 1, 1), (3, 1, 7), (4, 9, 1)])
def test_degenerate_networks_bitwise(G, cn, ncx, ncz):
    """One cell, one row or one column of cells; sources on the two far
    lattice corners and the same source twice in one call: every output
    bitwise against the oracle, duplicate rows identical."""
    C = _C()
    cls = tti_classes()
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b011)
    desc = C.cache_desc(n_dirs=360, modes=(0, 1))
    cache = G.import_cache(f, s, desc, 3)
    NX, NZ, _ = O.cell_lattice(ncx, ncz, cn)
    cid = layered_cells(ncx, ncz, cn, 3, 0)
    srcs = [0, NX * NZ - 1, 0]
    for mode in (0, 1):
        g = G.trace_cells(cache, desc, 3, ncx, ncz, cn, 10.0, 7.0, cid, mode, srcs)
        for si, src in enumerate(srcs):
            o = O.trace_cells_2d(ncx, ncz, cn, 10.0, 7.0, cid, f[:, mode], s[mode], src)
            for key in KEYS:
                assert np.array_equal(g[key][si], o[key]), (mode, si, key)
        for key in KEYS:
            assert np.array_equal(g[key][0], g[key][2])


def test_fluid_layer_blocks_shear_bitwise(G):
    """A fluid layer (no shear modulus) between two solids: qSV segments
    touching it have no cached entry (+inf weight), so the fluid nodes and
    the solid below them stay unreached while qP passes; every output
    bitwise against the oracle."""
    C = _C()
    solid = tti_classes(2)
    fluid = O.class_from_moduli(2.25e6, 2.25e6, 2.25e6, 0.0, 0.0, *[1000.0] * 5)
    cls = np.stack([solid[0], fluid, solid[1]])
    f, s = O.build_cache_2d(cls, n_dirs=360, mode_mask=0b011)
    desc = C.cache_desc(n_dirs=360, modes=(0, 1))
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncz, cn = 10, 9, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = layered_cells(ncx, ncz, cn, 3, 0)
    srcs = [NX // 2]
    for mode in (0, 1):
        g = G.trace_cells(cache, desc, 3, ncx, ncz, cn, 10.0, 10.0, cid, mode, srcs)
        o = O.trace_cells_2d(ncx, ncz, cn, 10.0, 10.0, cid, f[:, mode], s[mode], srcs[0])
        for key in KEYS:
            assert np.array_equal(g[key][0], o[key]), (mode, key)
        fl = (cid.reshape(-1) == 1) & mask.reshape(-1)
        if mode == 1:
            assert np.isinf(g["tauR"][0][fl]).all() and (g["predP"][0][fl] == -1).all()
        else:
            assert np.isfinite(g["tauR"][0][fl]).all()
