"""GPU parity of the slowness-sampled cache (eq 26 with the real slowness
angle as the cache index) and of traveltimes through it (the closest stored
ray direction per endpoint, text after eq 27, then eqs 28-31): the built
cache against the oracle's entries, traveltimes on imported oracle caches
bitwise (including random ray directions that exercise the lookup), and
the unsupported combinations rejected."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402
from test_oracle_slow import random_slow_cache  # noqa: E402


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import chert_gpu
    return chert_gpu


def _C():
    import paper_2609_26108_amd as C
    return C


def layered_classes():
    m = W.config2()
    return np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])


@pytest.mark.parametrize("n,reading", [(360, "mev"), (720, "mev"), (360, "oev"), (36, "oev")])
def test_cache_matches_oracle(G, n, reading):
    """Every mode of the layered model's classes, both readings of the
    inhomogeneity angle; entries 1e-10, statuses equal."""
    from test_gpu_cache import compare_cache
    C = _C()
    cls = layered_classes()
    kern = C.KERNEL_MEV if reading == "mev" else C.KERNEL_OEV
    desc = C.cache_desc(n_dirs=n, modes=(0, 1, 2), kernel=kern, sampling=C.SAMPLE_SLOWNESS)
    assert C.chert_build_cache_workspace_bytes(desc, cls.shape[0]) == 0
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    fg, sg = G.cache_to_numpy(cache, desc, cls.shape[0])
    fo, so = O.build_cache_slow_2d(cls, n=n, mode_mask=0b111,
                                   reading=O.MEV if reading == "mev" else O.OEV)
    st = compare_cache(fg, sg, fo, so, (0, 1, 2))
    print(n, reading, st, flush=True)
    # the stored theta_R is the sample's own angle, exactly
    q = np.arange(n)
    for m in range(3):
        ok = (so[m] & O.ST_NO_BRACKET) == 0
        assert np.array_equal(fg[5, m][ok], (q * (2 * np.pi / n))[None, :].repeat(
            cls.shape[0], 0)[ok])


def test_fluid_class(G):
    """A fluid class: shear columns FLUID with NaN fields, qP at V = Vp."""
    C = _C()
    c = O.class_from_moduli(2.25e6, 2.25e6, 2.25e6, 0.0, 0.0, *[1000.0] * 5)
    desc = C.cache_desc(n_dirs=72, modes=(0, 1, 2), sampling=C.SAMPLE_SLOWNESS)
    cache = G.build_cache(G.classes_from_arrays(c[None]), desc)
    fg, sg = G.cache_to_numpy(cache, desc, 1)
    fo, so = O.build_cache_slow_2d(c, n=72, mode_mask=0b111)
    np.testing.assert_array_equal(sg, so)
    assert np.all(np.isnan(fg[0, 1])) and np.all(np.isnan(fg[0, 2]))
    np.testing.assert_allclose(fg[0, 0], fo[0, 0], rtol=1e-12)


@pytest.mark.parametrize("launch", [0, 1])
@pytest.mark.parametrize("n,radius", [(360, 4), (720, 6), (72, 2)])
def test_trace_on_imported_cache_bitwise(G, n, radius, launch):
    """Traveltimes, t* and predecessors through an oracle-built slowness
    cache of the layered model (per-round and persistent launches) equal
    the oracle's Dijkstra bitwise."""
    C = _C()
    m = W.small_layered(nx=61, nz=41, radius=radius, seed=radius + n)
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    K = cls.shape[0]
    f, s = O.build_cache_slow_2d(cls, n=n, mode_mask=0b011)
    desc = C.cache_desc(n_dirs=n, modes=(0, 1), sampling=C.SAMPLE_SLOWNESS)
    cache = G.import_cache(f, s, desc, K)
    srcs = [m.sources[0], m.nx * m.nz - 1]
    for mode in (0, 1):
        g = G.trace(cache, desc, K, m.nx, m.nz, m.hx, m.hz, radius, m.class_id, mode, srcs,
                    launch=launch)
        for si, src in enumerate(srcs):
            o = O.trace_2d_slow(m.nx, m.nz, m.hx, m.hz, m.class_id, radius, f[:, mode],
                                s[mode], src)
            for key in ("tauR", "tauI", "tstar", "predP", "predA"):
                assert np.array_equal(g[key][si], o[key]), (mode, si, key)


@pytest.mark.parametrize("R,hx,hz", [(3, 10.0, 10.0), (5, 5.0, 7.5), (6, 12.5, 6.25)])
def test_trace_random_directions_bitwise(G, R, hx, hz):
    """Stored ray directions at random angles, some samples without a root:
    the closest-direction lookup picks a different column per endpoint
    class, so any disagreement with the oracle's lookup shows in the
    traveltimes or predecessors."""
    C = _C()
    rng = np.random.default_rng(R)
    K, n = 4, 90
    V, A, RX, RZ, st = random_slow_cache(K, n, rng)
    f = np.full((O.NF, 3, K, n), np.nan)
    s = np.zeros((3, K, n), np.int32)
    f[0, 0], f[1, 0], f[3, 0], f[4, 0] = V, A, RX, RZ
    s[0] = st
    nx, nz = 45, 37
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    desc = C.cache_desc(n_dirs=n, modes=(0,), sampling=C.SAMPLE_SLOWNESS)
    cache = G.import_cache(f, s, desc, K)
    srcs = [7, nx * nz // 2 + 3]
    g = G.trace(cache, desc, K, nx, nz, hx, hz, R, cid, 0, srcs)
    for si, src in enumerate(srcs):
        o = O.trace_2d_slow(nx, nz, hx, hz, cid, R, f[:, 0], s[0], src)
        for key in ("tauR", "tauI", "tstar", "predP", "predA"):
            assert np.array_equal(g[key][si], o[key]), (si, key)


def test_end_to_end_gpu_cache(G):
    """The GPU's own slowness cache of the layered model traced end to end
    against the oracle's cache and Dijkstra (1e-9)."""
    C = _C()
    m = W.small_layered(nx=81, nz=51, radius=5, seed=3)
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    K = cls.shape[0]
    desc = C.cache_desc(n_dirs=720, modes=(0, 1), sampling=C.SAMPLE_SLOWNESS)
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    fo, so = O.build_cache_slow_2d(cls, n=720, mode_mask=0b011)
    for mode in (0, 1):
        g = G.trace(cache, desc, K, m.nx, m.nz, m.hx, m.hz, 5, m.class_id, mode, m.sources[:1])
        o = O.trace_2d_slow(m.nx, m.nz, m.hx, m.hz, m.class_id, 5, fo[:, mode], so[mode],
                            m.sources[0])
        for key in ("tauR", "tauI", "tstar"):
            a, b = g[key][0], o[key]
            fin = np.isfinite(b)
            assert np.array_equal(np.isfinite(a), fin)
            rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
            assert rel.max() <= 1e-9, (mode, key, rel.max())


def test_unsupported_combinations(G):
    """Per-node grids, the node frontier and the surrogate start do not take
    slowness caches: UNSUPPORTED, nothing launched."""
    C = _C()
    cls = layered_classes()
    K = cls.shape[0]
    desc = C.cache_desc(n_dirs=72, modes=(0,), sampling=C.SAMPLE_SLOWNESS)
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    nx, nz = 20, 15
    out = torch.empty((1, nx * nz), dtype=torch.float64, device=G.DEV)
    # per-node grid (no class map)
    g = C.make_grid(nx, nz, 10.0, 10.0, 3, None)
    o = C.trace_opts(C.OUT_TAU_R)
    assert C.chert_trace_workspace_bytes(desc, K, g, 1, o) == 0
    # node frontier
    cid = torch.zeros(nx * nz, dtype=torch.int32, device=G.DEV)
    g = C.make_grid(nx, nz, 10.0, 10.0, 3, cid)
    o = C.trace_opts(C.OUT_TAU_R, launch=C.LAUNCH_FRONTIER)
    assert C.chert_trace_workspace_bytes(desc, K, g, 1, o) == 0
    # surrogate-started build (checked before the blob is looked at)
    with pytest.raises(C.ChertError) as e:
        C.chert_build_cache_surrogate(desc, G.classes_from_arrays(cls), K, cache, cache, cache)
    assert e.value.code == C.ERR_UNSUPPORTED
    # the tile path works on the same grid
    o = C.trace_opts(C.OUT_TAU_R)
    wsb = C.chert_trace_workspace_bytes(desc, K, g, 1, o)
    assert wsb > 0
    ws = torch.empty(wsb, dtype=torch.uint8, device=G.DEV)
    C.chert_trace_field(desc, cache, K, g, 0, [0], o, out, None, None, None, None, ws)
    torch.cuda.synchronize()
    assert out[0, 0].item() == 0.0 and torch.isfinite(out).all()
