"""GPU parity of the surrogate kernels (MLP on the matrix cores) against the
oracle's BF16 emulation and FP64 reference, and of the surrogate-started
cache build against the plain solver (GPU and oracle).

Bars: dataset and standardisation to FP32 rounding; forward 1e-3 relative
(FP32 accumulation order); gradients 1e-2 relative per parameter block;
Adam to FP32 rounding; surrogate-started caches equal to the plain cache
within the cache bar (1e-10 relative), so traveltimes agree far inside the
1e-4 relative bar asked of a surrogate form.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from oracle import surrogate as S  # noqa: E402
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


SHAPES = [shp for _, shp in S.SHAPES]


def new_blob(G, params):
    C = _C()
    lay = C.chert_surrogate_layout_of()
    assert lay.n_params == S.N_PARAMS and lay.n_in == S.N_IN and lay.n_out == S.N_OUT
    blob = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=G.DEV)
    assert blob.data_ptr() % 256 == 0
    C.chert_surrogate_init(blob, torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(G.DEV))
    return blob


def random_params(seed, bias_scale=0.1):
    p = W.mlp_init(SHAPES, seed)
    w = S.unpack(p)
    rng = np.random.default_rng(seed + 1)
    for name in ("b1", "b2", "b3", "b4"):
        w[name][:] = rng.normal(0, bias_scale, w[name].shape)
    return p


def blob_norm(blob):
    _, _, _, nrm = _C().surrogate_views(blob)
    n = nrm.cpu().numpy()
    return n[:16], n[16:32], n[32:36], n[36:40]


def standardise(blob, X, Y=None):
    mx, ix, my, sy = blob_norm(blob)
    Xs = ((X.astype(np.float32) - mx) * ix).astype(np.float32)
    if Y is None:
        return Xs
    return Xs, ((Y.astype(np.float32) - my) / sy).astype(np.float32)


def gpu_dataset(G, desc, cache, classes_dev, K):
    C = _C()
    n = bin(desc.mode_mask).count("1") * K * desc.n_cols
    x = torch.empty((n, 16), dtype=torch.float32, device=G.DEV)
    y = torch.empty((n, 4), dtype=torch.float32, device=G.DEV)
    ok = torch.empty(n, dtype=torch.int32, device=G.DEV)
    C.chert_surrogate_dataset(desc, cache, classes_dev, K, x, y, ok)
    torch.cuda.synchronize()
    return x, y, ok


def rock_classes(rock_table):
    cls = []
    for i, r in enumerate(rock_table):
        c = O.class_from_moduli(*(r[:5] * 1e6), *r[5:10])
        c[11] = math.radians([0.0, 25.0, -33.0, 71.5][i])
        cls.append(c)
    for L in W.config2().layers:
        cls.append(O.class_from_thomsen(*L.thomsen_args()))
    return np.stack(cls)


@pytest.mark.parametrize("subset", [False, True])
def test_dataset_reformats_cache(G, rock_table, subset):
    """Features and targets of every cache entry equal the oracle's
    reformatting of the same entries (FP64 arithmetic rounded to FP32)."""
    C = _C()
    cls = rock_classes(rock_table)
    sub = C.star_subset(5, 5.0, 5.0) if subset else None
    desc = C.cache_desc(modes=(0, 1, 2), subset=sub)
    cdev = G.classes_from_arrays(cls)
    cache = G.build_cache(cdev, desc)
    fg, sg = G.cache_to_numpy(cache, desc, cls.shape[0])
    x, y, ok = gpu_dataset(G, desc, cache, cdev, cls.shape[0])
    Xo, Yo, oko = S.dataset_from_cache(cls, fg, sg, subset=sub)
    assert np.array_equal(ok.cpu().numpy().astype(bool), oko)
    Xg = x.cpu().numpy()
    np.testing.assert_allclose(Xg, Xo.astype(np.float32), rtol=2.5e-7, atol=1e-7)
    Yg = y.cpu().numpy()[oko]
    np.testing.assert_allclose(Yg, Yo[oko].astype(np.float32), rtol=2.5e-7, atol=1e-9)


def test_fit_norm_matches_oracle(G):
    rng = np.random.default_rng(11)
    X = (rng.normal(2, 3, (5000, 16))).astype(np.float32)
    X[:, 10] = 1.0
    Y = rng.normal(-0.5, 0.2, (5000, 4)).astype(np.float32)
    ok = (rng.random(5000) < 0.8).astype(np.int32)
    blob = new_blob(G, random_params(1))
    C = _C()
    C.chert_surrogate_fit_norm(blob, torch.from_numpy(X).to(G.DEV), torch.from_numpy(Y).to(G.DEV),
                               torch.from_numpy(ok).to(G.DEV))
    torch.cuda.synchronize()
    mx, sx, my, sy = S.norm_stats(X.astype(np.float64), Y.astype(np.float64), ok.astype(bool))
    gm, gi, gym, gys = blob_norm(blob)
    np.testing.assert_allclose(gm, mx, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gi, 1.0 / sx, rtol=1e-6)
    np.testing.assert_allclose(gym, my, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gys, sy, rtol=1e-6)


def _fit_random_norm(G, blob, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.5, 2.0, (4000, 16)).astype(np.float32)
    Y = rng.normal(0.3, 1.5, (4000, 4)).astype(np.float32)
    ok = np.ones(4000, np.int32)
    _C().chert_surrogate_fit_norm(blob, torch.from_numpy(X).to(G.DEV),
                                  torch.from_numpy(Y).to(G.DEV), torch.from_numpy(ok).to(G.DEV))


@pytest.mark.parametrize("n", [1, 32, 1007])
def test_infer_matches_bf16_emulation(G, n):
    """Forward pass on the matrix cores = the oracle's BF16 emulation within
    1e-3 (relative to the output scale); ragged row counts."""
    C = _C()
    p = random_params(3)
    blob = new_blob(G, p)
    _fit_random_norm(G, blob, 4)
    rng = np.random.default_rng(5)
    X = rng.normal(0.5, 2.0, (n, 16)).astype(np.float32)
    y = torch.full((n, 4), np.nan, dtype=torch.float32, device=G.DEV)
    C.chert_surrogate_infer(blob, torch.from_numpy(X).to(G.DEV), y)
    torch.cuda.synchronize()
    Yg = y.cpu().numpy()
    _, _, my, sy = blob_norm(blob)
    o, _ = S.forward_bf16(p, standardise(blob, X))
    Ye = o * sy + my
    scale = np.abs(Ye).max(axis=0) + sy
    assert np.all(np.abs(Yg - Ye) <= 1e-3 * scale), np.abs(Yg - Ye).max(axis=0) / scale
    # and the FP64 network is within BF16 accuracy
    o64, _ = S.forward(p.astype(np.float64), standardise(blob, X).astype(np.float64))
    assert np.all(np.abs(Yg - (o64 * sy + my)) <= 3e-2 * scale)


def test_gradient_matches_bf16_emulation(G):
    """Loss and gradient of a ragged batch (100 samples: three full tiles
    and a partial one) against the BF16 emulation (1e-2 relative per
    parameter block) and the FP64 backward (cosine > 0.999)."""
    C = _C()
    p = random_params(6, 0.3)
    blob = new_blob(G, p)
    _fit_random_norm(G, blob, 7)
    rng = np.random.default_rng(8)
    X = rng.normal(0.5, 2.0, (500, 16)).astype(np.float32)
    Y = rng.normal(0.3, 1.5, (500, 4)).astype(np.float32)
    idx = rng.choice(500, 100, replace=False).astype(np.int32)
    grad = torch.empty(S.N_PARAMS, dtype=torch.float32, device=G.DEV)
    loss = torch.empty(1, dtype=torch.float32, device=G.DEV)
    ws = torch.empty(C.chert_surrogate_grad_workspace_bytes(100), dtype=torch.uint8, device=G.DEV)
    C.chert_surrogate_grad(blob, torch.from_numpy(X).to(G.DEV), torch.from_numpy(Y).to(G.DEV),
                           torch.from_numpy(idx).to(G.DEV), grad, loss, ws)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    Xs, Ys = standardise(blob, X[idx], Y[idx])
    Le, ge = S.backward_bf16(p, Xs, Ys)
    assert abs(float(loss.item()) - Le) <= 1e-3 * Le
    ge = ge.astype(np.float64)
    off = 0
    for name, shp in S.SHAPES:
        k = int(np.prod(shp))
        a, b = g[off:off + k], ge[off:off + k]
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), name
        off += k
    _, g64 = S.backward(p.astype(np.float64), Xs.astype(np.float64), Ys.astype(np.float64))
    assert g @ g64 / (np.linalg.norm(g) * np.linalg.norm(g64)) > 0.999


def test_adam_steps_match_oracle(G):
    """Two Adam steps on the FP32 master weights equal the oracle's update
    computed from the same gradients; the BF16 copies follow (the next
    forward pass equals the emulation with the new weights)."""
    C = _C()
    p = random_params(9)
    blob = new_blob(G, p)
    rng = np.random.default_rng(10)
    pv, mv, vv, _ = C.surrogate_views(blob)
    P, M, V = p.astype(np.float64), np.zeros(S.N_PARAMS), np.zeros(S.N_PARAMS)
    for t, lr in ((1, 1e-3), (2, 5e-4)):
        g = (rng.normal(0, 1, S.N_PARAMS) * 10.0 ** rng.uniform(-4, 0, S.N_PARAMS)).astype(np.float32)
        C.chert_surrogate_adam(blob, torch.from_numpy(g).to(G.DEV), t, lr)
        torch.cuda.synchronize()
        gd = g.astype(np.float64)
        # FP32 rounding bound: relative to the size of the terms of each
        # update (the result itself may cancel)
        m_scale = S.BETA1 * np.abs(M) + (1 - S.BETA1) * np.abs(gd)
        v_scale = S.BETA2 * V + (1 - S.BETA2) * gd * gd
        P0 = P
        P, M, V = S.adam(P, M, V, gd, t, lr)
        assert np.all(np.abs(mv.cpu().numpy() - M) <= 2e-6 * m_scale)
        assert np.all(np.abs(vv.cpu().numpy() - V) <= 2e-6 * v_scale)
        assert np.all(np.abs(pv.cpu().numpy() - P) <= 2e-6 * (np.abs(P0) + 10 * lr))
    X = rng.normal(0, 1, (64, 16)).astype(np.float32)
    y = torch.empty((64, 4), dtype=torch.float32, device=G.DEV)
    C.chert_surrogate_infer(blob, torch.from_numpy(X).to(G.DEV), y)
    torch.cuda.synchronize()
    o, _ = S.forward_bf16(pv.cpu().numpy(), X)
    assert np.abs(y.cpu().numpy() - o).max() <= 1e-3 * (np.abs(o).max() + 1)


def warm_build(G, classes_dev, desc, blob, K):
    C = _C()
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=G.DEV)
    ws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, K), dtype=torch.uint8,
                     device=G.DEV)
    stats = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=G.DEV)
    C.chert_build_cache_surrogate(desc, classes_dev, K, blob, cache, ws, stats)
    torch.cuda.synchronize()
    return cache, dict(zip(C.WARM_STATS, stats.cpu().numpy().tolist()))


def compare_to_plain(fw, sw, fp, sp, modes, tol=1e-10):
    """Warm entries against the plain GPU cache (same status, fields within
    tol; angles absolute)."""
    for m in modes:
        assert np.array_equal(sw[m], sp[m]), m
        ok = (sp[m] & (O.ST_NO_BRACKET | O.ST_FLUID)) == 0
        for fi, name in enumerate(O.FIELDS):
            a, b = fw[fi, m][ok], fp[fi, m][ok]
            if name in ("thR",):
                err = np.abs((a - b + np.pi) % (2 * np.pi) - np.pi)
            elif name in ("thI", "rx", "rz", "res"):
                err = np.abs(a - b)
                if name == "res":
                    assert np.all(a < 1e-11)
                    continue
            elif name == "Q":
                fin = np.isfinite(b)
                assert np.array_equal(np.isfinite(a), fin)
                err = np.where(fin, np.abs(a - b) / np.where(fin, np.abs(b), 1.0), 0.0)
            else:
                err = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
            assert np.all(err <= tol), (m, name, float(err.max()))


def test_untrained_surrogate_falls_back_to_plain(G):
    """A random (untrained) surrogate: whatever it predicts, the build
    equals the plain one (rejected jobs are re-solved by the plain path)."""
    C = _C()
    m = W.complex_2d(nx=24, nz=18, h=10.0, water_m=30.0, n_layers=5, n_faults=1, seed=5,
                     radius=3)
    rows = m.param_rows()
    params = torch.from_numpy(rows).to(G.DEV)
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(params, classes)
    desc = C.cache_desc(modes=(0, 1), n_sweep=720, subset=C.star_subset(3, m.hx, m.hz))
    plain = G.build_cache(classes, desc)
    blob = new_blob(G, random_params(12))
    warm, st = warm_build(G, classes, desc, blob, K)
    print("untrained", st)
    assert st["jobs"] == 2 * K
    fw, sw = G.cache_to_numpy(warm, desc, K)
    fp, sp = G.cache_to_numpy(plain, desc, K)
    compare_to_plain(fw, sw, fp, sp, (0, 1))


@pytest.fixture(scope="module")
def trained(G):
    """A surrogate trained on plain-solver entries of 400 seeded media over
    the full 1-degree direction set (3 modes: 432k entries)."""
    C = _C()
    rows = W.surrogate_training_rows(400, seed=W.seed_for(6))
    params = torch.from_numpy(rows).to(G.DEV)
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(params, classes)
    desc = C.cache_desc(modes=(0, 1, 2))
    cache = G.build_cache(classes, desc)
    x, y, ok = gpu_dataset(G, desc, cache, classes, K)
    blob = new_blob(G, W.mlp_init(SHAPES, seed=1))
    C.chert_surrogate_fit_norm(blob, x, y, ok)
    losses = C.train_surrogate(blob, x, y, ok, steps=3000, batch=1024, lr=2e-3, seed=2)
    torch.cuda.synchronize()
    L = losses.cpu().numpy()
    print("training loss first/last", L[:20].mean(), L[-200:].mean())
    return blob, L


def test_training_reduces_loss(trained):
    _, L = trained
    assert np.all(np.isfinite(L))
    assert L[-200:].mean() < 0.02 * L[:20].mean()


def test_trained_surrogate_build_matches_plain_and_oracle(G, trained):
    """Per-node caches of a small structurally complex model (media not in
    the training set), star subset, qP and qSV: the surrogate-started build
    equals the plain GPU build (1e-10) and the oracle (cache bar), and most
    jobs are served by the surrogate."""
    C = _C()
    from test_gpu_cache import compare_cache
    blob, _ = trained
    m = W.complex_2d(nx=40, nz=30, h=10.0, water_m=50.0, n_layers=8, n_faults=2, seed=21,
                     radius=5)
    rows = m.param_rows()
    params = torch.from_numpy(rows).to(G.DEV)
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(params, classes)
    sub = C.star_subset(5, m.hx, m.hz)
    desc = C.cache_desc(modes=(0, 1), subset=sub)
    plain = G.build_cache(classes, desc)
    warm, st = warm_build(G, classes, desc, blob, K)
    print("trained", st)
    fw, sw = G.cache_to_numpy(warm, desc, K)
    fp, sp = G.cache_to_numpy(plain, desc, K)
    compare_to_plain(fw, sw, fp, sp, (0, 1))
    assert st["fallback_jobs"] <= 0.5 * st["jobs"], st
    # oracle on a sample of nodes (every 7th)
    pick = np.arange(0, K, 7)
    cls_o = np.stack([O.class_from_thomsen(*r) for r in rows[pick]])
    fo, so = O.build_cache_2d(cls_o, mode_mask=0b011, subset=sub)
    compare_cache(fw[:, :, pick], sw[:, pick], fo, so, (0, 1))


def test_trained_surrogate_traveltimes(G, trained):
    """Traveltimes through surrogate-started and plain per-node caches agree
    (1e-4 relative is the bar for a surrogate form; they agree to the cache
    tolerance)."""
    C = _C()
    blob, _ = trained
    m = W.complex_2d(nx=48, nz=36, h=10.0, water_m=40.0, n_layers=8, n_faults=2, seed=22,
                     radius=5)
    rows = m.param_rows()
    params = torch.from_numpy(rows).to(G.DEV)
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(params, classes)
    desc = C.cache_desc(modes=(1,), subset=C.star_subset(5, m.hx, m.hz))
    plain = G.build_cache(classes, desc)
    warm, st = warm_build(G, classes, desc, blob, K)
    out = {}
    for name, cache in (("plain", plain), ("warm", warm)):
        out[name] = G.trace(cache, desc, K, m.nx, m.nz, m.hx, m.hz, 5, None, 1, m.sources,
                            outputs=C.OUT_TAU_R | C.OUT_TAU_I)
    a, b = out["warm"]["tauR"], out["plain"]["tauR"]
    fin = np.isfinite(b)
    assert np.array_equal(np.isfinite(a), fin)
    rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
    print("tau rel max", rel.max(), st)
    assert rel.max() <= 1e-4
    assert rel.max() <= 1e-9


def test_trained_surrogate_gain_over_plain(G, trained):
    """What the trained network buys: on the same per-node caches (9,600
    nodes, qSV, star bins) the surrogate-started build spends at least 4x
    less GPU time than the plain sweep-and-bracket build, with equal
    results (kernel time from HIP events around every library launch)."""
    C = _C()
    blob, _ = trained
    m = W.complex_2d(nx=120, nz=80, h=10.0, water_m=60.0, n_layers=10, n_faults=2, seed=23,
                     radius=5)
    rows = m.param_rows()
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(G.DEV), classes)
    desc = C.cache_desc(modes=(1,), subset=C.star_subset(5, m.hx, m.hz))
    G.build_cache(classes, desc)
    warm_build(G, classes, desc, blob, K)
    C.chert_prof_enable(True)
    plain = G.build_cache(classes, desc)
    t_plain = sum(v[1] for v in C.chert_prof_read().values())
    C.chert_prof_enable(True)
    warm, st = warm_build(G, classes, desc, blob, K)
    t_warm = sum(v[1] for v in C.chert_prof_read().values())
    C.chert_prof_enable(False)
    print(f"plain {t_plain:.3f} ms, surrogate-started {t_warm:.3f} ms, "
          f"gain {t_plain / t_warm:.1f}x", st)
    fw, sw = G.cache_to_numpy(warm, desc, K)
    fp, sp = G.cache_to_numpy(plain, desc, K)
    compare_to_plain(fw, sw, fp, sp, (1,))
    assert t_warm * 4.0 < t_plain


@pytest.mark.slow
def test_full_size_per_node_build_sampled(G, trained):
    """The structurally complex model at full size (1701 x 351 nodes, qSV,
    star bins): the surrogate-started per-node cache against the oracle's
    plain solve at 24 sampled solid nodes (every column), within the cache
    bar."""
    from test_gpu_cache import compare_cache
    C = _C()
    blob, _ = trained
    m = W.complex_2d()
    rows = m.param_rows()
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(G.DEV), classes)
    sub = C.star_subset(5, m.hx, m.hz)
    desc = C.cache_desc(modes=(1,), subset=sub)
    warm, st = warm_build(G, classes, desc, blob, K)
    print("full size", st)
    assert st["jobs"] == K
    f, s = C.cache_views(warm, desc, K)
    rng = np.random.default_rng(77)
    solid = np.flatnonzero(rows[:, 1] > 0)
    pick = np.sort(rng.choice(solid, 24, replace=False))
    idx = torch.from_numpy(pick).to(G.DEV)
    fg = f[:, :, idx].cpu().numpy()
    sg = s[:, idx].cpu().numpy()
    cls_o = np.stack([O.class_from_thomsen(*r) for r in rows[pick]])
    fo, so = O.build_cache_2d(cls_o, mode_mask=0b010, subset=sub)
    compare_cache(fg, sg, fo, so, (1,))


def _config5_classes(G, n=None):
    C = _C()
    m = W.config5(nx=8, ny=8, nz=8)
    rows = np.stack([[L.vp0, L.vs0, L.rho, L.eps, L.delta, L.gamma, L.tilt, L.azimuth, L.qp, L.qs]
                     for L in m.layers])
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(G.DEV), classes)
    return classes, K


def warm_build_3d(G, classes, desc, blob, K):
    C = _C()
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=G.DEV)
    ws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, K), dtype=torch.uint8,
                     device=G.DEV)
    stats = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=G.DEV)
    C.chert_build_cache_surrogate(desc, classes, K, blob, cache, ws, stats)
    torch.cuda.synchronize()
    return cache, dict(zip(C.WARM_STATS, stats.cpu().numpy().tolist()))


def test_warm_3d_full_direction_set_matches_plain(G, trained):
    """The surrogate-started 3D cache of the layered 3D model's six classes
    on all 41,253 Fibonacci directions (qP, qSV): every entry has the plain
    3D build's status and fields within 1e-10, most directions accepted from
    the Newton polish; sampled entries also against the oracle's solve at
    the direction's polar angle to the axis."""
    C = _C()
    blob, _ = trained
    classes, K = _config5_classes(G)
    N = O.N_FIB
    desc = C.cache_desc(dim=3, n_dirs=N, modes=(0, 1))
    plain = G.build_cache(classes, desc)
    warm, st = warm_build_3d(G, classes, desc, blob, K)
    print("3D warm", st, flush=True)
    assert st["jobs"] == 2 * K and st["directions"] == 2 * K * N
    assert st["fallback_jobs"] < 0.2 * st["directions"]
    fw, sw = G.cache_to_numpy(warm, desc, K)
    fp, sp = G.cache_to_numpy(plain, desc, K)
    compare_to_plain(fw, sw, fp, sp, (0, 1))
    cls = classes.cpu().numpy()
    fib = O.fibonacci(N)
    rng = np.random.default_rng(31)
    for _ in range(24):
        k, mode, i = int(rng.integers(K)), int(rng.integers(2)), int(rng.integers(N))
        t0, p0 = cls[k, 11], cls[k, 12]
        ez = np.array([np.sin(t0) * np.cos(p0), np.sin(t0) * np.sin(p0), np.cos(t0)])
        f, so = O.solve(cls[k], mode, np.arccos(np.clip(fib[i] @ ez, -1, 1)))
        assert sw[mode, k, i] == so
        if so & (O.ST_NO_BRACKET | O.ST_FLUID):
            continue
        for name in ("V", "A"):
            assert abs(fw[O.FIELDS.index(name), mode, k, i] - f[name]) <= 1e-10 * abs(f[name])


def test_warm_3d_untrained_surrogate_equals_plain(G):
    """A random (untrained) surrogate in 3D: directions its polish cannot
    take go to the plain search; the cache equals the plain build."""
    C = _C()
    classes, K = _config5_classes(G)
    desc = C.cache_desc(dim=3, n_dirs=3000, modes=(0, 1), n_sweep=720)
    plain = G.build_cache(classes, desc)
    warm, st = warm_build_3d(G, classes, desc, new_blob(G, random_params(5)), K)
    print("3D untrained", st, flush=True)
    assert st["fallback_jobs"] > 0
    fw, sw = G.cache_to_numpy(warm, desc, K)
    fp, sp = G.cache_to_numpy(plain, desc, K)
    compare_to_plain(fw, sw, fp, sp, (0, 1))
