"""GPU parity at the settings of the angular-step and star-radius ablations
(angular sampling 0.5, 1, 2 and 10 degrees; forward-star radius 2 to 6):
caches against the oracle's at every step, traveltimes on imported caches
bitwise (class caches and per-node caches on the star's bins, including the
2-degree step where diagonal edges fall half-way between two tabulated
directions)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import chert_gpu
    return chert_gpu


def _C():
    import paper_2609_26108_amd as C
    return C


@pytest.mark.parametrize("n_dirs", [720, 180, 36])
def test_cache_at_angular_steps(G, n_dirs):
    """Class caches of the layered model at 0.5, 2 and 10 degrees, all modes,
    against the oracle (1e-10)."""
    from test_gpu_cache import compare_cache
    C = _C()
    m = W.config2()
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    desc = C.cache_desc(n_dirs=n_dirs, modes=(0, 1, 2), n_sweep=1440)
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    fg, sg = G.cache_to_numpy(cache, desc, cls.shape[0])
    fo, so = O.build_cache_2d(cls, n_dirs=n_dirs, mode_mask=0b111)
    st = compare_cache(fg, sg, fo, so, (0, 1, 2))
    print(n_dirs, st, flush=True)


@pytest.mark.parametrize("n_dirs,radius", [(720, 6), (180, 2), (180, 6), (36, 4), (720, 3)])
def test_class_trace_at_step_and_radius(G, n_dirs, radius):
    """Traveltimes, t* and predecessors on an imported class cache at the
    ablation's steps and radii equal the oracle's bitwise."""
    C = _C()
    m = W.small_layered(nx=61, nz=41, radius=radius, seed=radius + n_dirs)
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    f, s = O.build_cache_2d(cls, n_dirs=n_dirs, mode_mask=0b011, n_sweep=720)
    desc = C.cache_desc(n_dirs=n_dirs, modes=(0, 1), n_sweep=720)
    K = cls.shape[0]
    cache = G.import_cache(f, s, desc, K)
    srcs = [m.sources[0], m.nx * m.nz - 1]
    for mode in (0, 1):
        g = G.trace(cache, desc, K, m.nx, m.nz, m.hx, m.hz, radius, m.class_id, mode, srcs)
        for si, src in enumerate(srcs):
            o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, radius, f[0, mode], f[1, mode],
                           s[mode], src, n_dirs=n_dirs)
            for key in ("tauR", "tauI", "tstar", "predP", "predA"):
                assert np.array_equal(g[key][si], o[key]), (mode, si, key)


@pytest.mark.parametrize("n_dirs,radius", [(180, 5), (720, 6), (36, 3), (180, 2)])
def test_per_node_trace_at_step_and_radius(G, n_dirs, radius):
    """Per-node caches on the star's bins at 2, 0.5 and 10 degrees: pushes
    read an edge's weight from the tail's row at the reversed offset, which
    needs bin(-o) = bin(o) + n_dirs/2 exactly (the 2-degree diagonals are
    half-step ties); every field and predecessor equals the oracle's."""
    C = _C()
    m = W.complex_2d(nx=41, nz=29, h=10.0, water_m=40.0, n_layers=6, n_faults=1, seed=9,
                     radius=radius, modes=(0, 1))
    rows = m.param_rows()
    cls = np.stack([O.class_from_thomsen(*r) for r in rows])
    sub = O.star_subset(radius, m.hx, m.hz, n_dirs)
    assert np.array_equal(sub, C.star_subset(radius, m.hx, m.hz, n_dirs))
    f, s = O.build_cache_2d(cls, n_dirs=n_dirs, mode_mask=0b011, n_sweep=360, subset=sub)
    desc = C.cache_desc(n_dirs=n_dirs, modes=(0, 1), n_sweep=360, subset=sub)
    N = rows.shape[0]
    cache = G.import_cache(f, s, desc, N)
    for mode in (0, 1):
        g = G.trace(cache, desc, N, m.nx, m.nz, m.hx, m.hz, radius, None, mode, m.sources)
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, None, radius, f[0, mode], f[1, mode], s[mode],
                       m.sources[0], n_dirs=n_dirs, subset=sub)
        for key in ("tauR", "tauI", "tstar", "predP", "predA"):
            assert np.array_equal(g[key][0], o[key]), (mode, key)


@pytest.mark.parametrize("n_dirs,radius", [(720, 6), (180, 5)])
def test_per_node_gpu_cache_at_step(G, n_dirs, radius):
    """The GPU's own per-node cache on the star's bins at 0.5 and 2 degrees
    against the oracle's entries (1e-10), then traced end to end (1e-9)."""
    from test_gpu_cache import compare_cache
    C = _C()
    m = W.complex_2d(nx=33, nz=21, h=10.0, water_m=30.0, n_layers=4, n_faults=1, seed=13,
                     radius=radius, modes=(1,))
    rows = m.param_rows()
    N = rows.shape[0]
    classes = torch.empty((N, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(G.DEV), classes)
    sub = C.star_subset(radius, m.hx, m.hz, n_dirs)
    desc = C.cache_desc(n_dirs=n_dirs, modes=(1,), n_sweep=720, subset=sub)
    cache = G.build_cache(classes, desc)
    fg, sg = G.cache_to_numpy(cache, desc, N)
    cls = np.stack([O.class_from_thomsen(*r) for r in rows])
    fo, so = O.build_cache_2d(cls, n_dirs=n_dirs, mode_mask=0b010, n_sweep=720, subset=sub)
    compare_cache(fg, sg, fo, so, (1,))
    g = G.trace(cache, desc, N, m.nx, m.nz, m.hx, m.hz, radius, None, 1, m.sources)
    o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, None, radius, fo[0, 1], fo[1, 1], so[1],
                   m.sources[0], n_dirs=n_dirs, subset=sub)
    for key in ("tauR", "tauI", "tstar"):
        a, b = g[key][0], o[key]
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin)
        rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
        assert rel.max() <= 1e-9, (key, rel.max())
