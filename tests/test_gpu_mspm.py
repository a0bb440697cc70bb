"""GPU parity of the MSPM baseline (Algorithm 1 on the cell network, no
cache: every visited cell's corners solved afresh at the exact segment
directions, non-corner nodes reconstructed from the corners of their edge)
against the oracle's MSPM form: traveltimes and t* within 1e-9 (the solves
agree with the oracle's to about 1e-12), predecessor trees complete, and
the isotropic medium equal to the cached network."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from test_oracle_mspm import two_classes  # noqa: E402


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import chert_gpu
    return chert_gpu


def _C():
    import paper_2609_26108_amd as C
    return C


def close(a, b, tol=1e-9):
    fin = np.isfinite(b)
    assert np.array_equal(np.isfinite(a), fin)
    rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
    assert rel.max(initial=0.0) <= tol, rel.max()
    return rel.max(initial=0.0)


@pytest.mark.parametrize("mode,kernel,bucket,cn", [(0, 0, 0.0, 4), (1, 0, 16.0, 4), (1, 1, 0.0, 3),
                                                   (2, 0, 4.0, 5), (0, 0, 0.0, 1)])
def test_mspm_matches_oracle(G, mode, kernel, bucket, cn):
    C = _C()
    cls = two_classes()
    ncx, ncz = 8, 6
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    # a tilted band of the second class that cuts through cells
    X, Z = np.meshgrid(np.arange(NX), np.arange(NZ))
    cid = np.where((Z + 0.3 * X).reshape(-1) > 0.55 * NZ, 1, 0).astype(np.int32)
    src = int(np.flatnonzero(mask.reshape(-1))[5])
    st = C.TraceStats()
    g = G.trace_mspm(cls, ncx, ncz, cn, 10.0, 8.0, cid, mode, [src], bucket_width=bucket,
                     kernel=kernel, n_sweep=720, stats=st)
    o = O.trace_mspm_2d(ncx, ncz, cn, 10.0, 8.0, cid, cls, mode, src, reading=kernel, n_sweep=720)
    for key in ("tauR", "tauI", "tstar"):
        print(key, close(g[key][0], o[key]), flush=True)
    node = mask.reshape(-1)
    for key in ("predP", "predA"):
        p = g[key][0]
        assert p[src] == -1 and np.all(p[node & (np.arange(node.size) != src)] >= 0)
        assert np.all(p[~node] == -1)
    # every visit solved its four corners along every canonical direction
    assert st.edge_relaxations[1] == 4 * st.tile_visits[0] * 2 * cn * (cn + 1)


def test_isotropic_equals_cached_network(G):
    C = _C()
    c = O.class_from_thomsen(3000.0, 1700.0, 2300, 0.0, 0.0, 0.0, 0.0, 0, np.inf, np.inf)
    ncx, ncz, cn = 10, 7, 5
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = np.zeros(NX * NZ, np.int32)
    g = G.trace_mspm(c[None], ncx, ncz, cn, 10.0, 10.0, cid, 0, [25], n_sweep=720)
    f, s = O.build_cache_2d(c, n_dirs=360, mode_mask=0b001, n_sweep=720)
    desc = C.cache_desc(n_dirs=360, modes=(0,), n_sweep=720)
    cache = G.import_cache(f, s, desc, 1)
    h = G.trace_cells(cache, desc, 1, ncx, ncz, cn, 10.0, 10.0, cid, 0, [25])
    node = mask.reshape(-1)
    close(g["tauR"][0][node], h["tauR"][0][node], 1e-13)
    assert np.all(g["tauI"][0][node] == 0.0)


def test_mspm_argument_checks(G):
    C = _C()
    cls = G.classes_from_arrays(two_classes())
    ncx, ncz, cn = 4, 3, 4
    NX, NZ, mask = O.cell_lattice(ncx, ncz, cn)
    cid = torch.zeros(NX * NZ, dtype=torch.int32, device=G.DEV)
    g = C.make_cell_grid(ncx, ncz, cn, 10.0, 10.0, cid)
    o = C.trace_opts(C.OUT_TAU_R)
    out = torch.full((1, NX * NZ), -3.0, dtype=torch.float64, device=G.DEV)
    ws = torch.empty(C.chert_trace_mspm_workspace_bytes(2, g, 1, o), dtype=torch.uint8,
                     device=G.DEV)
    for kw in ({"kernel": 7}, {"n_sweep": 4}, {"n_sweep": 8192}):
        with pytest.raises(C.ChertError) as e:
            C.chert_trace_mspm(cls, 2, g, 0, [0], o, out, workspace_dev=ws, **kw)
        assert e.value.code == C.ERR_INVALID_ARG
    with pytest.raises(C.ChertError):
        C.chert_trace_mspm(cls, 2, g, 3, [0], o, out, workspace_dev=ws)
    torch.cuda.synchronize()
    assert torch.all(out == -3.0)
