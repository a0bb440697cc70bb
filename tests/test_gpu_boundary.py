"""GPU checks of the C ABI's failure surface: build counters
(chert_cache_stats), the solver's residual cap and step cap (NOCONV
entries), the caller's abort word, and a bad class map that leaves every
output untouched.  Every kernel exits normally in each case; failures are
forced from the host (a preset abort word, a step cap of one)."""
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


def host_counts(f, s, modes):
    """chert_cache_stats recomputed on the host from the status and
    residual arrays of the built modes."""
    st = np.concatenate([s[m].reshape(-1) for m in modes])
    res = np.concatenate([f[7, m].reshape(-1) for m in modes])
    rooted = (st & (O.ST_NO_BRACKET | O.ST_FLUID)) == 0
    r = np.abs(res[rooted])
    r = r[~np.isnan(r)]
    return {"n_entries": st.size, "n_converged": int(np.sum((st & ~O.ST_ILL) == 0)),
            "n_noconv": int(np.sum((st & 16) != 0)), "n_illcond": int(np.sum((st & O.ST_ILL) != 0)),
            "n_nobracket": int(np.sum((st & O.ST_NO_BRACKET) != 0)),
            "n_unusable": int(np.sum((st & (O.ST_FLUID | O.ST_NONPHYS)) != 0)),
            "max_resid": float(r.max()) if r.size else 0.0}


def built_with_stats(G, classes, desc_kw, K):
    C = _C()
    stats = torch.full((C.CACHE_STATS_BYTES,), 0xAB, dtype=torch.uint8, device=G.DEV)
    desc = C.cache_desc(stats=stats, **desc_kw)
    cache = G.build_cache(classes, desc)
    return desc, cache, C.cache_stats_of(stats).as_dict()


@pytest.mark.parametrize("case", ["layered", "rock_fluid", "3d"])
def test_cache_stats_match_status_arrays(G, rock_table, case):
    """The build's device counters equal the counts of the status array it
    wrote; with the default tolerance no entry is NOCONV and the largest
    residual is far below it."""
    C = _C()
    if case == "layered":
        m = W.config2()
        classes = G.classes_from_layers(m.layers)
        kw = dict(n_dirs=360, modes=(0, 1, 2))
    elif case == "rock_fluid":
        from workloads import Layer
        layers = W.small_layered(seed=4).layers
        layers[0] = Layer(1500.0, 0.0, 1000.0, 0.0, 0.0, 0.0, 0.0, 1000.0, 1000.0)
        classes = G.classes_from_layers(layers)
        kw = dict(n_dirs=360, modes=(0, 1, 2), n_sweep=720)
    else:
        m = W.config5()
        classes = G.classes_from_layers(m.layers[:2])
        kw = dict(dim=3, n_dirs=4000, modes=(0, 1), n_sweep=720)
    K = classes.shape[0]
    desc, cache, st = built_with_stats(G, classes, kw, K)
    f, s = G.cache_to_numpy(cache, desc, K)
    want = host_counts(f, s, kw["modes"])
    print(case, st, flush=True)
    for k, v in want.items():
        if k == "max_resid":
            assert st[k] == pytest.approx(v, rel=0, abs=0), k
        else:
            assert st[k] == v, k
    assert st["n_fallback"] == 0 and st["n_noconv"] == 0
    assert st["max_resid"] < 1e-11


def test_step_cap_marks_noconv_and_trace_avoids_it(G):
    """max_iter = 1 stops each bracket's refinement after one Newton step and
    one halving: the roots miss the residual cap, the entries carry NOCONV,
    the counters say so, and the trace treats them as unusable exactly as
    the oracle's Dijkstra does on the same imported statuses."""
    C = _C()
    m = W.small_layered(nx=40, nz=28, radius=3, seed=7)
    classes = G.classes_from_layers(m.layers)
    K = classes.shape[0]
    kw = dict(n_dirs=360, modes=(0, 1), n_sweep=720, max_iter=1, resid_tol=1e-12)
    desc, cache, st = built_with_stats(G, classes, kw, K)
    f, s = G.cache_to_numpy(cache, desc, K)
    want = host_counts(f, s, (0, 1))
    print(st, flush=True)
    assert st["n_noconv"] == want["n_noconv"] > 0
    assert st["n_converged"] == want["n_converged"]
    assert np.all(f[7][(s & 16) != 0] > 1e-12)
    for mode in (0, 1):
        g = G.trace(cache, desc, K, m.nx, m.nz, m.hx, m.hz, m.radius, m.class_id, mode, m.sources)
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, f[0, mode], f[1, mode],
                       s[mode], m.sources[0])
        for key in ("tauR", "tauI", "tstar", "predP", "predA"):
            assert np.array_equal(g[key][0], o[key]), key


def test_surrogate_build_reports_fallback_entries(G):
    """An untrained surrogate sends jobs back to the plain solver; the
    build's counters give those jobs' entries as n_fallback, in agreement
    with the warm-start counters."""
    C = _C()
    from test_gpu_surrogate import new_blob, random_params
    m = W.complex_2d(nx=24, nz=18, h=10.0, water_m=30.0, n_layers=5, n_faults=1, seed=5,
                     radius=3)
    rows = m.param_rows()
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(G.DEV), classes)
    sub = C.star_subset(3, m.hx, m.hz)
    stats = torch.zeros(C.CACHE_STATS_BYTES, dtype=torch.uint8, device=G.DEV)
    desc = C.cache_desc(modes=(0, 1), n_sweep=720, subset=sub, stats=stats)
    blob = new_blob(G, random_params(12))
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=G.DEV)
    ws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, K), dtype=torch.uint8,
                     device=G.DEV)
    wst = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=G.DEV)
    C.chert_build_cache_surrogate(desc, classes, K, blob, cache, ws, wst)
    torch.cuda.synchronize()
    st = C.cache_stats_of(stats).as_dict()
    warm = dict(zip(C.WARM_STATS, wst.cpu().numpy().tolist()))
    print(st, warm, flush=True)
    assert warm["fallback_jobs"] > 0
    assert st["n_fallback"] == warm["fallback_jobs"] * len(sub)
    f, s = G.cache_to_numpy(cache, desc, K)
    want = host_counts(f, s, (0, 1))
    for k in ("n_entries", "n_converged", "n_noconv", "n_illcond", "n_nobracket", "n_unusable"):
        assert st[k] == want[k], k


# ------------------------------------------------------------ bad class map


def _uneven_batch(G, bad=False):
    C = _C()
    from test_gpu_trace import uneven_batch
    b, jobs, keep = uneven_batch(G)
    if bad:  # one out-of-range class id in the second grid's map
        cid = keep[5]
        cid[7] = 1000
        torch.cuda.synchronize()
    return C, b, jobs, keep


@pytest.mark.parametrize("launch", [0, 1, 2])
def test_bad_class_map_leaves_outputs_untouched(G, launch):
    """A class id out of range: INVALID_ARG and every output keeps the
    caller's contents, on the tiles (per-round and persistent launches) and
    on the node frontier."""
    C, b, jobs, keep = _uneven_batch(G, bad=True)
    for j in jobs:
        for t in j[5].values():
            t.fill_(-5)
    opts = C.trace_opts(C.OUT_ALL, launch=launch)
    ws = torch.empty(C.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_batch(b, opts, ws)
    assert e.value.code == C.ERR_INVALID_ARG
    torch.cuda.synchronize()
    for j in jobs:
        for k, t in j[5].items():
            assert bool((t == -5).all()), k


@pytest.mark.parametrize("launch", [0, 1])
def test_bad_class_map_graph_leaves_outputs_untouched(G, launch):
    """The same inside a replayed graph: finish reports INVALID_ARG and the
    outputs keep their contents."""
    C, b, jobs, keep = _uneven_batch(G, bad=True)
    opts = C.trace_opts(C.OUT_ALL, launch=launch, max_rounds=64 if launch == 0 else 0)
    ws = torch.empty(C.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = C.TraceGraph(b, opts, ws, stream=stream)
    try:
        for j in jobs:
            for t in j[5].values():
                t.fill_(-5)
        torch.cuda.synchronize()
        graph.launch(stream)
        with pytest.raises(C.ChertError) as e:
            graph.finish(None, stream)
        assert e.value.code == C.ERR_INVALID_ARG
        torch.cuda.synchronize()
        for j in jobs:
            for k, t in j[5].items():
                assert bool((t == -5).all()), k
    finally:
        graph.close()


# --------------------------------------------------------------- abort word


def _abort_word(value):
    w = torch.zeros(1, dtype=torch.int32).pin_memory()
    w[0] = value
    return w


def _upper_bounds(jobs):
    """tau_R and tau_I of an aborted run: +inf or at least the oracle's
    value (each is the length of some path); the source itself is 0."""
    for mdl, f, s, mode, srcs, out in jobs:
        tr = out["tau_r"].cpu().numpy()
        ti = out["tau_i"].cpu().numpy()
        for si, src in enumerate(srcs):
            o = O.trace_2d(mdl.nx, mdl.nz, mdl.hx, mdl.hz, mdl.class_id, mdl.radius,
                           f[0, mode], f[1, mode], s[mode], src)
            for a, b in ((tr[si], o["tauR"]), (ti[si], o["tauI"])):
                assert a[src] == 0.0
                assert np.all(a >= b), int(np.sum(a < b))


@pytest.mark.parametrize("launch", [0, 1, 2])
def test_preset_abort_word_returns_aborted(G, launch):
    """A raised abort word: the eager call returns ABORTED on the tiles
    (host check after the first launches; the kernels stop visiting tiles
    once workgroup 0 has seen the word) and on the node frontier, and the
    traveltimes are valid upper bounds."""
    C, b, jobs, keep = _uneven_batch(G)
    word = _abort_word(1)
    opts = C.trace_opts(C.OUT_ALL, launch=launch, abort_flag=word)
    ws = torch.empty(C.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_batch(b, opts, ws)
    assert e.value.code == C.ERR_ABORTED, e.value
    torch.cuda.synchronize()
    _upper_bounds(jobs)


@pytest.mark.parametrize("launch", [0, 1])
def test_preset_abort_word_in_graph(G, launch):
    """The graph forms poll the word on the device (per-round launches: each
    round; persistent: at every device-wide barrier): finish returns
    ABORTED; a later replay with the word lowered gives the oracle's fields
    bitwise."""
    C, b, jobs, keep = _uneven_batch(G)
    from test_gpu_trace import check_batch
    word = _abort_word(1)
    opts = C.trace_opts(C.OUT_ALL, launch=launch, abort_flag=word,
                        max_rounds=96 if launch == 0 else 0)
    ws = torch.empty(C.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = C.TraceGraph(b, opts, ws, stream=stream)
    try:
        graph.launch(stream)
        with pytest.raises(C.ChertError) as e:
            graph.finish(None, stream)
        assert e.value.code == C.ERR_ABORTED, e.value
        torch.cuda.synchronize()
        _upper_bounds(jobs)
        word[0] = 0
        graph.launch(stream)
        graph.finish(None, stream)
        torch.cuda.synchronize()
        check_batch(jobs)
    finally:
        graph.close()


@pytest.mark.parametrize("launch", [0, 1, 2])
def test_lowered_abort_word_changes_nothing(G, launch):
    """An abort word that stays 0 is polled but the fields are the oracle's
    bitwise."""
    C, b, jobs, keep = _uneven_batch(G)
    from test_gpu_trace import check_batch
    word = _abort_word(0)
    opts = C.trace_opts(C.OUT_ALL, launch=launch, abort_flag=word)
    ws = torch.empty(C.chert_trace_batch_workspace_bytes(b, opts), dtype=torch.uint8,
                     device=G.DEV)
    C.chert_trace_batch(b, opts, ws)
    torch.cuda.synchronize()
    check_batch(jobs)

