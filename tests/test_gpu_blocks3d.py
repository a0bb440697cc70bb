"""GPU parity of the block network (the cell network in 3D: nodes on block
faces, every face-point pair of a block a segment; eqs 27-31 with the
Fibonacci cache of eq 35): traveltimes, t* and predecessors through the C
ABI against the oracle's node Dijkstra, bitwise on imported oracle caches
(block edges of 1 to 3 intervals, unordered and block-ordered rounds, a
batch of sources), at the compact 3D TTI size, the GPU's own 3D cache traced
end to end, and the error paths."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

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


def tti3_classes(K=3):
    return np.stack([O.class_from_thomsen(3000.0 + 400 * k, 1700.0 + 200 * k, 2300, 0.1 * k,
                                          0.05 * k, 0.08, math.radians(25.0), 0.9 * k - 0.5,
                                          60.0 + 20 * k, 40.0 + 10 * k) for k in range(K)])


def banded(NX, NY, NZ, K, seed):
    """Class per lattice point by undulating depth band."""
    rng = np.random.default_rng(seed)
    z = np.arange(NZ)[:, None, None]
    x = np.arange(NX)[None, None, :]
    y = np.arange(NY)[None, :, None]
    u = 1.5 * np.sin(x * rng.uniform(0.2, 0.6) + y * rng.uniform(0.1, 0.5))
    return np.clip(((z + u) * K) // NZ, 0, K - 1).astype(np.int32)


def face_sources(ncx, ncy, ncz, cn, picks):
    NX, NY, NZ, mask = O.block_lattice(ncx, ncy, ncz, cn)
    nodes = np.flatnonzero(mask.reshape(-1))
    return [int(nodes[int(p * (nodes.size - 1))]) for p in picks]


@pytest.fixture(scope="module")
def small_cache():
    f, s = O.build_cache_3d(tti3_classes(), N=400, mode_mask=0b011)
    return f, s


@pytest.mark.parametrize("cn,nc,bucket", [(3, (4, 3, 4), 0.0), (3, (4, 3, 4), 4.0),
                                          (2, (6, 4, 5), 0.0), (2, (5, 5, 3), 16.0),
                                          (1, (9, 6, 7), 0.0), (1, (7, 4, 6), 2.0)])
def test_imported_cache_bitwise(G, small_cache, cn, nc, bucket):
    """Imported oracle 3D cache of three tilted TTI classes with azimuths in
    undulating bands; both modes, two sources in one batch; every output
    bitwise."""
    C = _C()
    f, s = small_cache
    desc = C.cache_desc(n_dirs=400, modes=(0, 1), dim=3)
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncy, ncz = nc
    NX, NY, NZ, _ = O.block_lattice(ncx, ncy, ncz, cn)
    cid = banded(NX, NY, NZ, 3, cn)
    srcs = face_sources(ncx, ncy, ncz, cn, (0.05, 0.6))
    h = (10.0, 12.5, 8.0)
    for mode in (0, 1):
        st = C.TraceStats()
        g = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, *h, cid, mode, srcs,
                           bucket_width=bucket, stats=st)
        assert st.rounds[0] > 0 and st.tile_visits[0] > 0 and st.rounds[1] > 0
        for si, src in enumerate(srcs):
            o = O.trace_blocks_3d(ncx, ncy, ncz, cn, *h, cid, f[0, mode], f[1, mode], s[mode],
                                  src, N=400)
            for key in KEYS:
                assert np.array_equal(g[key][si], o[key]), (mode, si, key)
        # the reported BFS depth is the deepest predecessor tree of the call
        deepest = max(tree_levels(g[k][si], src) for si, src in enumerate(srcs)
                      for k in ("predP", "predA"))
        assert st.rounds[1] == deepest, (st.rounds[1], deepest)


def random_cache(K, N, rng):
    """A cache of independent random entries per (class, direction): any
    segment that reads a different column than the oracle's changes its
    weight, so the traveltimes show a wrong closest-direction pick."""
    f = np.full((O.NF, 3, K, N), np.nan)
    s = np.zeros((3, K, N), np.int32)
    for m in (0, 1):
        f[0, m] = rng.uniform(1500.0, 4500.0, (K, N))
        f[1, m] = rng.uniform(0.0, 2e-5, (K, N))
    return f, s


def test_compact_3d_tti_full_size(G):
    """The compact 3D TTI block model (18 x 18 x 4 blocks of 160 m, block
    edges of 3 intervals, 55 x 55 x 13 lattice, 4 undulating layers) with a
    random cache of the full 41253 Fibonacci directions (every column a
    different value, so the closest-direction pick over all of them is
    checked): the centre source, both fields, every output bitwise against
    the oracle's Dijkstra, and the raypaths to the 361 surface receivers."""
    C = _C()
    m = W.blocks_3d()
    K = len(m.layers)
    f, s = random_cache(K, m.n_dirs, np.random.default_rng(41253))
    desc = C.cache_desc(n_dirs=m.n_dirs, modes=(0, 1), dim=3)
    cache = G.import_cache(f, s, desc, K)
    for mode in (0, 1):
        st = C.TraceStats()
        g = G.trace_blocks(cache, desc, K, m.ncx, m.ncy, m.ncz, m.block_n, m.h, m.h, m.h,
                           m.class_id, mode, m.sources, bucket_width=4.0, stats=st)
        print("mode", mode, "rounds", st.rounds[0], "levels", st.rounds[1], "visits",
              st.tile_visits[0], flush=True)
        o = O.trace_blocks_3d(m.ncx, m.ncy, m.ncz, m.block_n, m.h, m.h, m.h, m.class_id,
                              f[0, mode], f[1, mode], s[mode], m.sources[0], N=m.n_dirs)
        for key in KEYS:
            assert np.array_equal(g[key][0], o[key]), (mode, key)
        _, _, _, mask = O.block_lattice(m.ncx, m.ncy, m.ncz, m.block_n)
        assert np.isfinite(g["tauR"][0][mask.reshape(-1)]).all()
        # raypaths (eqs 25, 33-34) to the 361 surface receivers from the
        # GPU's predecessors equal the oracle's from its own, segment by
        # segment, for both fields
        src = m.sources[0]
        for key in ("predP", "predA"):
            for rcv in m.receivers:
                path = C.chert_extract_raypath(g[key][0], src, rcv)
                rc, ref = O.raypath(o[key], src, rcv)
                assert rc == 0 and np.array_equal(path, ref), (mode, key, rcv)
                assert path[0] == src and path[-1] == rcv


def test_gpu_cache_end_to_end(G):
    """The GPU's own 3D cache of the tilted classes traced end to end
    against the oracle's cache and Dijkstra (1e-9 relative)."""
    C = _C()
    cls = tti3_classes()
    N = 2000
    desc = C.cache_desc(n_dirs=N, modes=(0, 1), dim=3)
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    fo, so = O.build_cache_3d(cls, N=N, mode_mask=0b011)
    ncx, ncy, ncz, cn = 5, 4, 4, 3
    NX, NY, NZ, _ = O.block_lattice(ncx, ncy, ncz, cn)
    cid = banded(NX, NY, NZ, 3, 9)
    srcs = face_sources(ncx, ncy, ncz, cn, (0.3,))
    for mode in (0, 1):
        g = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, 10.0, 10.0, 10.0, cid, mode, srcs)
        o = O.trace_blocks_3d(ncx, ncy, ncz, cn, 10.0, 10.0, 10.0, cid, fo[0, mode], fo[1, mode],
                              so[mode], srcs[0], N=N)
        for key in ("tauR", "tauI", "tstar"):
            a, b = g[key][0], o[key]
            fin = np.isfinite(b)
            assert np.array_equal(np.isfinite(a), fin)
            rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
            assert rel.max() <= 1e-9, (mode, key, rel.max())


def test_outputs_subset_and_fields(G, small_cache):
    """tau_I alone, and tau_R with its tree but no t*: the computed outputs
    equal the full call's."""
    C = _C()
    f, s = small_cache
    desc = C.cache_desc(n_dirs=400, modes=(0, 1), dim=3)
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncy, ncz, cn = 3, 3, 3, 2
    NX, NY, NZ, _ = O.block_lattice(ncx, ncy, ncz, cn)
    cid = banded(NX, NY, NZ, 3, 4)
    srcs = face_sources(ncx, ncy, ncz, cn, (0.5,))
    full = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, 10, 10, 10, cid, 1, srcs)
    a = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, 10, 10, 10, cid, 1, srcs,
                       outputs=C.OUT_TAU_I)
    assert np.array_equal(a["tauI"], full["tauI"])
    b = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, 10, 10, 10, cid, 1, srcs,
                       outputs=C.OUT_TAU_R | C.OUT_PRED_P)
    assert np.array_equal(b["tauR"], full["tauR"]) and np.array_equal(b["predP"], full["predP"])


def test_errors(G, small_cache):
    """A 2D cache, block_n beyond 3, a source inside a block, a class id out
    of range: INVALID_ARG before any output is written."""
    C = _C()
    f, s = small_cache
    desc3 = C.cache_desc(n_dirs=400, modes=(0, 1), dim=3)
    cache = G.import_cache(f, s, desc3, 3)
    ncx, ncy, ncz, cn = 2, 2, 2, 3
    NX, NY, NZ, _ = O.block_lattice(ncx, ncy, ncz, cn)
    n = NX * NY * NZ
    cid = torch.zeros(n, dtype=torch.int32, device=G.DEV)
    o = C.trace_opts(C.OUT_TAU_R)
    g = C.make_block_grid(ncx, ncy, ncz, cn, 10.0, 10.0, 10.0, cid)
    desc2 = C.cache_desc(n_dirs=360, modes=(0, 1))
    assert C.chert_trace_blocks_workspace_bytes(desc2, 3, g, 1, o) == 0
    g4 = C.make_block_grid(ncx, ncy, ncz, 4, 10.0, 10.0, 10.0, cid)
    assert C.chert_trace_blocks_workspace_bytes(desc3, 3, g4, 1, o) == 0
    wsb = C.chert_trace_blocks_workspace_bytes(desc3, 3, g, 1, o)
    assert wsb > 0
    ws = torch.empty(wsb, dtype=torch.uint8, device=G.DEV)
    out = torch.full((1, n), -7.0, dtype=torch.float64, device=G.DEV)
    inside = 1 + NX * (1 + NY * 1)
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_blocks(desc3, cache, 3, g, 0, [inside], o, out, None, None, None, None, ws)
    assert e.value.code == C.ERR_INVALID_ARG
    cid[5] = 3
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_blocks(desc3, cache, 3, g, 0, [0], o, out, None, None, None, None, ws)
    assert e.value.code == C.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert (out == -7.0).all()


@pytest.mark.parametrize("cn,nc", [(1, (1, 1, 1)), (3, (1, 1, 1)), (2, (1, 5, 1)), (3, (4, 1, 2))])
def test_degenerate_networks_bitwise(G, small_cache, cn, nc):
    """One block, one row of blocks along y, one layer of blocks; sources on
    the two far lattice corners and the same source twice in one call: every
    output bitwise against the oracle, duplicate rows identical."""
    C = _C()
    f, s = small_cache
    desc = C.cache_desc(n_dirs=400, modes=(0, 1), dim=3)
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncy, ncz = nc
    NX, NY, NZ, _ = O.block_lattice(ncx, ncy, ncz, cn)
    cid = banded(NX, NY, NZ, 3, 2)
    srcs = [0, NX * NY * NZ - 1, 0]
    for mode in (0, 1):
        g = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, 9.0, 11.0, 10.0, cid, mode, srcs)
        for si, src in enumerate(srcs):
            o = O.trace_blocks_3d(ncx, ncy, ncz, cn, 9.0, 11.0, 10.0, cid, f[0, mode], f[1, mode],
                                  s[mode], src, N=400)
            for key in KEYS:
                assert np.array_equal(g[key][si], o[key]), (mode, si, key)
        for key in KEYS:
            assert np.array_equal(g[key][0], g[key][2])


def test_fluid_layer_blocks_shear_bitwise(G):
    """A fluid layer between two tilted solids: qSV weights touching it are
    +inf, so its nodes and the solid below stay unreached; qP passes.  Every
    output bitwise against the oracle."""
    C = _C()
    solid = tti3_classes(2)
    fluid = O.class_from_moduli(2.25e6, 2.25e6, 2.25e6, 0.0, 0.0, *[1000.0] * 5)
    cls = np.stack([solid[0], fluid, solid[1]])
    f, s = O.build_cache_3d(cls, N=400, mode_mask=0b011)
    desc = C.cache_desc(n_dirs=400, modes=(0, 1), dim=3)
    cache = G.import_cache(f, s, desc, 3)
    ncx, ncy, ncz, cn = 4, 3, 6, 2
    NX, NY, NZ, mask = O.block_lattice(ncx, ncy, ncz, cn)
    z = np.arange(NZ)[:, None, None]
    cid = np.broadcast_to(np.clip(z * 3 // NZ, 0, 2), (NZ, NY, NX)).astype(np.int32).copy()
    srcs = [NX // 2 + NX * (NY // 2)]
    for mode in (0, 1):
        g = G.trace_blocks(cache, desc, 3, ncx, ncy, ncz, cn, 10.0, 10.0, 10.0, cid, mode, srcs)
        o = O.trace_blocks_3d(ncx, ncy, ncz, cn, 10.0, 10.0, 10.0, cid, f[0, mode], f[1, mode],
                              s[mode], srcs[0], N=400)
        for key in KEYS:
            assert np.array_equal(g[key][0], o[key]), (mode, key)
        fl = (cid.reshape(-1) == 1) & mask.reshape(-1)
        if mode == 1:
            assert np.isinf(g["tauR"][0][fl]).all() and (g["predP"][0][fl] == -1).all()
        else:
            assert np.isfinite(g["tauR"][0][fl]).all()
