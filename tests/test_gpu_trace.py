"""GPU parity of the traveltime fields (chert_trace_field) against the
oracle's Dijkstra.

On an imported (oracle-computed) cache the fields must be bitwise equal
(tau_R, tau_I, t*) and the predecessors identical: both sides compute the
minimum over paths of the left-to-right FP64 sum of identical weights.
End to end (GPU cache -> GPU trace vs oracle cache -> oracle Dijkstra) the bar
is 1e-9 relative.
"""
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


def C():
    import paper_2609_26108_amd as mod
    return mod


def oracle_cache(model, modes, n_sweep=1440):
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in model.layers])
    mask = sum(1 << m for m in modes)
    f, s = O.build_cache_2d(cls, n_dirs=model.n_dirs, mode_mask=mask, n_sweep=n_sweep)
    return cls, f, s


def assert_fields_equal(g, o, s_idx=0):
    for key in ("tauR", "tauI", "tstar"):
        if g[key] is None:
            continue
        a, b = g[key][s_idx], o[key]
        assert np.array_equal(a, b), (key, int(np.sum(a != b)))
    for key in ("predP", "predA"):
        if g[key] is None:
            continue
        a, b = g[key][s_idx], o[key]
        assert np.array_equal(a, b), (key, int(np.sum(a != b)))


def imported_case(G, model, modes, tile=(0, 0), sources=None, n_sweep=1440, launch=0,
                  bucket=0.0, group=0):
    cls, f, s = oracle_cache(model, modes, n_sweep)
    Cm = C()
    desc = Cm.cache_desc(n_dirs=model.n_dirs, modes=modes, n_sweep=n_sweep)
    K = cls.shape[0]
    cache = G.import_cache(f, s, desc, K)
    sources = model.sources if sources is None else sources
    for mode in modes:
        g = G.trace(cache, desc, K, model.nx, model.nz, model.hx, model.hz, model.radius,
                    model.class_id, mode, sources, tile_x=tile[0], tile_z=tile[1],
                    launch=launch, bucket_width=bucket, push_group=group)
        for si, src in enumerate(sources):
            o = O.trace_2d(model.nx, model.nz, model.hx, model.hz, model.class_id,
                           model.radius, f[0, mode], f[1, mode], s[mode], src)
            print(f"mode {mode} src {src}: finite {int(np.isfinite(o['tauR']).sum())}", flush=True)
            assert_fields_equal(g, o, si)


@pytest.mark.parametrize("launch,bucket", [(0, 0.0), (1, 0.0), (0, 4.0), (1, 16.0), (2, 0.0),
                                           (2, 8.0)])
def test_imported_cache_small_layered_bitwise(G, launch, bucket):
    """Every launch form (one launch per round; one persistent launch per
    phase; either with tiles visited in key order; the node frontier with one
    bucket or near/far buckets) reaches the oracle's fields bitwise."""
    m = W.small_layered()
    imported_case(G, m, (0, 1, 2), launch=launch, bucket=bucket)


@pytest.mark.parametrize("tile,bucket", [((8, 8), 0.0), ((16, 4), 0.0), ((32, 16), 0.0),
                                         ((64, 16), 0.0), ((8, 8), 2.0), ((16, 4), 32.0)])
def test_tile_shapes_give_identical_fields(G, tile, bucket):
    """Determinism across schedules: every tile shape and ordering width
    reaches the same bits."""
    m = W.small_layered(nx=53, nz=29, radius=4, seed=3)
    imported_case(G, m, (1,), tile=tile, bucket=bucket)


@pytest.mark.parametrize("group,launch", [(1, 0), (4, 1), (8, 0), (8, 1)])
def test_push_groups_give_identical_fields(G, group, launch):
    """Every push-group width (offsets per push work item), per-round and
    persistent, on class caches, reaches the oracle's bits."""
    m = W.small_layered(nx=47, nz=31, radius=5, seed=8)
    imported_case(G, m, (0, 1), tile=(16, 16), group=group, launch=launch)


def test_multiple_sources_one_call(G):
    m = W.small_layered(nx=41, nz=27, radius=2, seed=5)
    srcs = [0, m.nx * m.nz - 1, 17 + m.nx * 13, 40]
    imported_case(G, m, (0,), sources=srcs)


@pytest.mark.parametrize("launch", [0, 2])
def test_degenerate_grids(G, launch):
    """One-row and one-column grids, a 1x1 grid, radius 1 and radius 8, on
    the tiles and on the node frontier."""
    for nx, nz, R in [(57, 1, 3), (1, 45, 2), (1, 1, 1), (19, 17, 8), (33, 2, 1)]:
        m = W.small_layered(nx=nx, nz=nz, radius=R, seed=nx + nz)
        m.sources = [min(m.sources[0], nx * nz - 1)]
        imported_case(G, m, (0,), n_sweep=360, launch=launch)


@pytest.mark.parametrize("launch", [0, 2])
def test_fluid_region_blocks_shear(G, launch):
    """A class without shear stiffness: shear-mode edges into it are
    impassable (tau = inf, pred = -1), qP passes."""
    m = W.small_layered(nx=30, nz=20, radius=3, seed=11)
    from workloads import Layer
    m.layers[0] = Layer(1500.0, 0.0, 1000.0, 0.0, 0.0, 0.0, 0.0, 1000.0, 1000.0)
    imported_case(G, m, (0, 1), n_sweep=360, launch=launch)


def test_end_to_end_config1(G):
    """Config 1 at full size: GPU cache + GPU trace vs the oracle (1e-9)."""
    m = W.config1()
    Cm = C()
    desc = Cm.cache_desc(n_dirs=360, modes=m.modes)
    cache = G.build_cache(G.classes_from_layers(m.layers), desc)
    cls, f, s = oracle_cache(m, m.modes)
    for mode in m.modes:
        g = G.trace(cache, desc, 1, m.nx, m.nz, m.hx, m.hz, m.radius, m.class_id, mode, m.sources)
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, f[0, mode], f[1, mode],
                       s[mode], m.sources[0])
        for key in ("tauR", "tauI", "tstar"):
            a, b = g[key][0], o[key]
            fin = np.isfinite(b)
            assert np.array_equal(np.isfinite(a), fin)
            rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
            assert rel.max() <= 1e-9, (key, rel.max())


@pytest.mark.parametrize("launch", [0, 2])
def test_end_to_end_config2_full_size(G, launch):
    """Config 2 (401 x 201, radius 5, 5 classes, 3 modes) end to end, on the
    tiles and on the node frontier."""
    m = W.config2()
    Cm = C()
    desc = Cm.cache_desc(n_dirs=360, modes=m.modes)
    cache = G.build_cache(G.classes_from_layers(m.layers), desc)
    cls, f, s = oracle_cache(m, m.modes)
    for mode in m.modes:
        g = G.trace(cache, desc, len(m.layers), m.nx, m.nz, m.hx, m.hz, m.radius, m.class_id,
                    mode, m.sources, launch=launch)
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, f[0, mode], f[1, mode],
                       s[mode], m.sources[0])
        for key in ("tauR", "tauI", "tstar"):
            a, b = g[key][0], o[key]
            fin = np.isfinite(b)
            assert np.array_equal(np.isfinite(a), fin)
            rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
            print(mode, key, float(rel.max()), flush=True)
            assert rel.max() <= 1e-9, (key, rel.max())


@pytest.mark.parametrize("launch", [0, 2])
def test_invalid_class_id_reported(G, launch):
    m = W.small_layered(nx=20, nz=10, radius=2, seed=1)
    cls, f, s = oracle_cache(m, (0,), n_sweep=360)
    Cm = C()
    desc = Cm.cache_desc(n_dirs=360, modes=(0,), n_sweep=360)
    cache = G.import_cache(f, s, desc, cls.shape[0])
    cid = m.class_id.copy()
    cid[3, 4] = 99
    with pytest.raises(Cm.ChertError) as e:
        G.trace(cache, desc, cls.shape[0], m.nx, m.nz, m.hx, m.hz, m.radius, cid, 0, m.sources,
                launch=launch)
    assert e.value.code == 1


def uneven_batch(G):
    """Two grids of different size and class count, two modes each, several
    sources, on imported oracle caches."""
    import torch
    Cm = C()
    m1 = W.small_layered(nx=61, nz=35, radius=3, seed=21)
    m2 = W.small_layered(nx=29, nz=47, n_layers=4, radius=3, seed=22)
    jobs = []
    b = Cm.Batch()
    keep = []
    for mdl, srcs in ((m1, [0, 61 * 35 - 1, 30 + 61 * 17]), (m2, [5, 28 + 29 * 40])):
        cls, f, s = oracle_cache(mdl, (0, 1), n_sweep=720)
        K = cls.shape[0]
        desc = Cm.cache_desc(n_dirs=360, modes=(0, 1), n_sweep=720)
        cache = G.import_cache(f, s, desc, K)
        cid = torch.from_numpy(mdl.class_id.reshape(-1).astype(np.int32)).to(G.DEV)
        grid = Cm.make_grid(mdl.nx, mdl.nz, mdl.hx, mdl.hz, mdl.radius, cid)
        for mode in (0, 1):
            n = mdl.n_nodes
            out = dict(tau_r=torch.empty((len(srcs), n), dtype=torch.float64, device=G.DEV),
                       tau_i=torch.empty((len(srcs), n), dtype=torch.float64, device=G.DEV),
                       tstar=torch.empty((len(srcs), n), dtype=torch.float64, device=G.DEV),
                       pred_p=torch.empty((len(srcs), n), dtype=torch.int32, device=G.DEV),
                       pred_a=torch.empty((len(srcs), n), dtype=torch.int32, device=G.DEV))
            b.add(desc, cache, K, grid, mode, srcs, **out)
            jobs.append((mdl, f, s, mode, srcs, out))
        keep += [cache, cid, grid, desc]
    return b, jobs, keep


def check_batch(jobs):
    for mdl, f, s, mode, srcs, out in jobs:
        g = {"tauR": out["tau_r"].cpu().numpy(), "tauI": out["tau_i"].cpu().numpy(),
             "tstar": out["tstar"].cpu().numpy(), "predP": out["pred_p"].cpu().numpy(),
             "predA": out["pred_a"].cpu().numpy()}
        for si, src in enumerate(srcs):
            o = O.trace_2d(mdl.nx, mdl.nz, mdl.hx, mdl.hz, mdl.class_id, mdl.radius,
                           f[0, mode], f[1, mode], s[mode], src)
            assert_fields_equal(g, o, si)


@pytest.mark.parametrize("launch,bucket", [(0, 0.0), (1, 0.0), (0, 8.0), (1, 64.0), (2, 0.0),
                                           (2, 16.0)])
def test_batch_uneven_grids_modes_sources_bitwise(G, launch, bucket):
    """chert_trace_batch over uneven grids, modes and sources: every field
    bitwise equal to the oracle, in every launch form."""
    Cm = C()
    b, jobs, keep = uneven_batch(G)
    stats = Cm.TraceStats()
    opts = Cm.trace_opts(Cm.OUT_ALL, launch=launch, stats=stats, bucket_width=bucket)
    ws = torch.empty(Cm.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    Cm.chert_trace_batch(b, opts, ws)
    torch.cuda.synchronize()
    print("launch", launch, "bucket", bucket, stats.as_dict())
    assert stats.rounds[0] > 0 and stats.rounds[1] > 0
    if launch != Cm.LAUNCH_FRONTIER:  # the tree phase computes predecessors and t* together
        assert stats.rounds[2] == 0 and stats.tile_visits[1] > 0
    check_batch(jobs)


@pytest.mark.parametrize("launch,bucket", [(1, 0.0), (1, 16.0), (0, 0.0), (0, 16.0)])
def test_graph_replays_match_eager(G, launch, bucket):
    """The batch captured as one graph (persistent phases, or per-round
    launches with a round budget from an eager run): three replays, each
    after eager work of the program's own and a wipe of the outputs, equal
    the eager run bitwise (and so the oracle), with or without tile
    ordering."""
    Cm = C()
    b, jobs, keep = uneven_batch(G)
    budget = 0
    if launch == Cm.LAUNCH_PER_ROUND:
        st = Cm.TraceStats()
        o0 = Cm.trace_opts(Cm.OUT_ALL, bucket_width=bucket, stats=st)
        w0 = torch.empty(Cm.chert_trace_batch_workspace_bytes(b, o0), dtype=torch.uint8,
                         device=G.DEV)
        Cm.chert_trace_batch(b, o0, w0)
        torch.cuda.synchronize()
        budget = max(st.rounds) + 8
        del w0
    opts = Cm.trace_opts(Cm.OUT_ALL, launch=launch, bucket_width=bucket, max_rounds=budget)
    ws = torch.empty(Cm.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    Cm.chert_trace_batch(b, opts, ws)
    torch.cuda.synchronize()
    eager = [{k: v.clone() for k, v in j[5].items()} for j in jobs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = Cm.TraceGraph(b, opts, ws, stream=stream)
    try:
        for rep in range(3):
            x = torch.randn(256, 256, device=G.DEV)
            y = (x @ x).sum()
            torch.cuda.synchronize()
            assert torch.isfinite(y)
            for j in jobs:
                for t in j[5].values():
                    t.fill_(-7)
            torch.cuda.synchronize()
            graph.launch(stream)
            stats = Cm.TraceStats()
            graph.finish(stats, stream)
            assert stats.rounds[0] > 0 and stats.rounds[1] > 0, stats.as_dict()
            for j, ref in zip(jobs, eager):
                for k, v in j[5].items():
                    assert torch.equal(v, ref[k]), (rep, k)
    finally:
        graph.close()
    check_batch(jobs)


def test_graph_short_round_budget_reports_no_convergence(G):
    """A per-round graph whose round budget is too short finishes with
    NO_CONVERGENCE (every kernel still exits normally)."""
    Cm = C()
    b, jobs, keep = uneven_batch(G)
    opts = Cm.trace_opts(Cm.OUT_ALL, launch=Cm.LAUNCH_PER_ROUND, max_rounds=2)
    ws = torch.empty(Cm.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = Cm.TraceGraph(b, opts, ws, stream=stream)
    try:
        graph.launch(stream)
        with pytest.raises(Cm.ChertError) as e:
            graph.finish(Cm.TraceStats(), stream)
        assert e.value.code == 4, e.value
    finally:
        graph.close()


def test_autotuned_options_give_identical_fields(G):
    """The autotuner picks one of its candidates; the full batch traced with
    the picked options is still bitwise the oracle's."""
    Cm = C()
    b, jobs, keep = uneven_batch(G)
    opts = Cm.trace_opts(Cm.OUT_ALL)
    ws = torch.empty(Cm.chert_trace_autotune_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    ms = Cm.chert_trace_autotune(b, opts, ws)
    print("autotuned", opts.tile_x, opts.tile_z, opts.push_group, opts.launch, opts.bucket_width,
          ms)
    assert ms > 0 and opts.launch in (0, 1, 2)
    if opts.launch == Cm.LAUNCH_FRONTIER:
        assert opts.bucket_width in (16.0, 64.0)
    else:
        assert opts.push_group in (1, 2, 4, 8) and opts.tile_x * opts.tile_z <= 1024
        assert opts.bucket_width in (0.0, 16.0, 64.0, 256.0)
    for j in jobs:
        for t in j[5].values():
            t.fill_(-3)
    Cm.chert_trace_batch(b, opts, ws)
    torch.cuda.synchronize()
    check_batch(jobs)


@pytest.mark.parametrize("launch,bucket,group", [(0, 0.0, 0), (0, 8.0, 0), (1, 32.0, 0),
                                                 (2, 0.0, 0), (2, 16.0, 0), (0, 0.0, 8),
                                                 (1, 0.0, 4), (0, 0.0, 1)])
def test_per_node_trace_bitwise(G, launch, bucket, group):
    """Per-node cache (no class map): GPU traveltimes and predecessors on an
    imported oracle cache are bitwise the oracle's, on the tiles and on the
    node frontier."""
    import torch
    Cm = C()
    m = W.complex_2d(nx=45, nz=33, h=10.0, water_m=60.0, n_layers=8, n_faults=2, seed=5,
                     radius=3, modes=(0, 1))
    rows = m.param_rows()
    cls = np.stack([O.class_from_thomsen(*r) for r in rows])
    sub = O.star_subset(3, m.hx, m.hz)
    f, s = O.build_cache_2d(cls, mode_mask=0b011, n_sweep=360, subset=sub)
    desc = Cm.cache_desc(modes=(0, 1), n_sweep=360, subset=sub)
    N = rows.shape[0]
    cache = G.import_cache(f, s, desc, N)
    for mode in (0, 1):
        n = m.n_nodes
        out = dict(tau_r=torch.empty((1, n), dtype=torch.float64, device=G.DEV),
                   tau_i=torch.empty((1, n), dtype=torch.float64, device=G.DEV),
                   tstar=torch.empty((1, n), dtype=torch.float64, device=G.DEV),
                   pred_p=torch.empty((1, n), dtype=torch.int32, device=G.DEV),
                   pred_a=torch.empty((1, n), dtype=torch.int32, device=G.DEV))
        grid = Cm.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, None)
        opts = Cm.trace_opts(Cm.OUT_ALL, launch=launch, bucket_width=bucket, push_group=group)
        ws = torch.empty(Cm.chert_trace_workspace_bytes(desc, N, grid, 1, opts),
                         dtype=torch.uint8, device=G.DEV)
        Cm.chert_trace_field(desc, cache, N, grid, mode, m.sources, opts, workspace_dev=ws, **out)
        torch.cuda.synchronize()
        g = {"tauR": out["tau_r"].cpu().numpy(), "tauI": out["tau_i"].cpu().numpy(),
             "tstar": out["tstar"].cpu().numpy(), "predP": out["pred_p"].cpu().numpy(),
             "predA": out["pred_a"].cpu().numpy()}
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, None, m.radius, f[0, mode], f[1, mode], s[mode],
                       m.sources[0], subset=sub)
        print(f"mode {mode}: finite {int(np.isfinite(o['tauR']).sum())}", flush=True)
        assert_fields_equal(g, o, 0)


def test_lean_builds_many_tiles_bitwise(G):
    """A batch with more than 8 tiles per compute unit (8 x 8 tiles over a
    200 x 96 grid, five sources, tau_R and tau_I problems: 3000 tiles) runs
    the occupancy-limited kernel builds; fields, t* and predecessors still
    equal the oracle's bitwise."""
    m = W.small_layered(nx=200, nz=96, radius=3)
    srcs = [0, 99, 200 * 50 + 100, 200 * 95 + 199, 200 * 20 + 30]
    imported_case(G, m, (0,), tile=(8, 8), sources=srcs)


def test_lean_builds_per_node_many_sources_bitwise(G):
    """Per-node cache, 35 sources on one grid with 8 x 8 tiles (2 x 35 x 30 =
    2100 tiles: the occupancy-limited builds on the per-node weight path);
    every source's fields and predecessors equal the oracle's bitwise."""
    import torch
    Cm = C()
    m = W.complex_2d(nx=45, nz=33, h=10.0, water_m=60.0, n_layers=8, n_faults=2, seed=5,
                     radius=3, modes=(0, 1))
    rows = m.param_rows()
    cls = np.stack([O.class_from_thomsen(*r) for r in rows])
    sub = O.star_subset(3, m.hx, m.hz)
    f, s = O.build_cache_2d(cls, mode_mask=0b001, n_sweep=360, subset=sub)
    desc = Cm.cache_desc(modes=(0,), n_sweep=360, subset=sub)
    N = rows.shape[0]
    cache = G.import_cache(f, s, desc, N)
    n = m.n_nodes
    srcs = [int(v) for v in np.linspace(0, n - 1, 35).astype(np.int64)]
    S = len(srcs)
    out = dict(tau_r=torch.empty((S, n), dtype=torch.float64, device=G.DEV),
               tau_i=torch.empty((S, n), dtype=torch.float64, device=G.DEV),
               tstar=torch.empty((S, n), dtype=torch.float64, device=G.DEV),
               pred_p=torch.empty((S, n), dtype=torch.int32, device=G.DEV),
               pred_a=torch.empty((S, n), dtype=torch.int32, device=G.DEV))
    grid = Cm.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, None)
    opts = Cm.trace_opts(Cm.OUT_ALL, tile_x=8, tile_z=8)
    ws = torch.empty(Cm.chert_trace_workspace_bytes(desc, N, grid, S, opts), dtype=torch.uint8,
                     device=G.DEV)
    Cm.chert_trace_field(desc, cache, N, grid, 0, srcs, opts, workspace_dev=ws, **out)
    torch.cuda.synchronize()
    g = {"tauR": out["tau_r"].cpu().numpy(), "tauI": out["tau_i"].cpu().numpy(),
         "tstar": out["tstar"].cpu().numpy(), "predP": out["pred_p"].cpu().numpy(),
         "predA": out["pred_a"].cpu().numpy()}
    for si, src in enumerate(srcs):
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, None, m.radius, f[0, 0], f[1, 0], s[0], src,
                       subset=sub)
        assert_fields_equal(g, o, si)


@pytest.mark.parametrize("tile,n_src", [((32, 32), 64), ((8, 8), 32)])
def test_list_mode_bitwise(G, tile, n_src):
    """A batch with more tiles than four times the resident workgroups (64
    sources x 2 fields x 20 tiles of 32 x 32 = 2560; or 32 x 2 x 320 tiles
    of 8 x 8 = 20,480, one wavefront each, more than four times 20 resident
    per compute unit): the per-round launches walk each round's list of
    active tiles (tau by ticket, from counters a workgroup of any size
    clears) instead of one workgroup per tile.  Eager and as a replayed
    graph, every field, t* and predecessor equals the oracle's bitwise."""
    Cm = C()
    m = W.small_layered(nx=160, nz=128, radius=3, seed=31)
    cls, f, s = oracle_cache(m, (0,), n_sweep=720)
    K = cls.shape[0]
    desc = Cm.cache_desc(n_dirs=360, modes=(0,), n_sweep=720)
    cache = G.import_cache(f, s, desc, K)
    rng = np.random.default_rng(77)
    srcs = sorted(rng.choice(m.n_nodes, n_src, replace=False).tolist())
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(G.DEV)
    grid = Cm.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, cid)
    n, S = m.n_nodes, len(srcs)
    out = {k: torch.empty((S, n), dtype=torch.float64, device=G.DEV)
           for k in ("tau_r", "tau_i", "tstar")}
    out.update({k: torch.empty((S, n), dtype=torch.int32, device=G.DEV)
                for k in ("pred_p", "pred_a")})
    b = Cm.Batch()
    b.add(desc, cache, K, grid, 0, srcs, **out)
    st = Cm.TraceStats()
    opts = Cm.trace_opts(Cm.OUT_ALL, tile[0], tile[1], stats=st)
    ws = torch.empty(Cm.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    Cm.chert_trace_batch(b, opts, ws)
    torch.cuda.synchronize()
    print(st.as_dict(), flush=True)
    eager = {k: v.clone() for k, v in out.items()}
    gopts = Cm.trace_opts(Cm.OUT_ALL, tile[0], tile[1], max_rounds=max(st.rounds) + 8)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = Cm.TraceGraph(b, gopts, ws, stream=stream)
    try:
        for rep in range(2):
            for t in out.values():
                t.fill_(-4)
            torch.cuda.synchronize()
            graph.launch(stream)
            graph.finish(None, stream)
            torch.cuda.synchronize()
            for k, v in out.items():
                assert torch.equal(v, eager[k]), (rep, k)
    finally:
        graph.close()
    g = {"tauR": eager["tau_r"].cpu().numpy(), "tauI": eager["tau_i"].cpu().numpy(),
         "tstar": eager["tstar"].cpu().numpy(), "predP": eager["pred_p"].cpu().numpy(),
         "predA": eager["pred_a"].cpu().numpy()}
    for si in range(0, S, 7):
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, f[0, 0], f[1, 0], s[0],
                       srcs[si])
        assert_fields_equal(g, o, si)
