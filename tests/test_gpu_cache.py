"""GPU parity of the cache builder (chert_build_cache) against the CPU oracle.

Bar: cache quantities within 1e-10 relative (angles within 1e-10 rad), status
codes equal.  Entries flagged ILL_CONDITIONED (|dpsi/dtheta_R| < 1e-2 at the
chosen root) are compared separately with 1e-6 and counted.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

KM2 = 1e6


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import chert_gpu
    return chert_gpu


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def compare_cache(fg, sg, fo, so, modes, tol=1e-10, tol_ill=1e-6, res_tol=1e-11):
    """fields [NF][3][K][D]; returns stats dict; asserts the bar."""
    stats = {"entries": 0, "ill": 0, "max_rel": 0.0}
    for m in modes:
        np.testing.assert_array_equal(sg[m] & ~O.ST_ILL, so[m] & ~O.ST_ILL)
        ok = (so[m] & O.ST_NO_BRACKET) == 0
        ok &= (so[m] & O.ST_FLUID) == 0
        # NOCONV entries hold the refinement's last iterate, not a root:
        # only their status is compared
        blank = ~ok
        ok &= (so[m] & O.ST_NOCONV) == 0
        stats["noconv"] = stats.get("noconv", 0) + int(((so[m] & O.ST_NOCONV) != 0).sum())
        ill = ((so[m] | sg[m]) & O.ST_ILL) != 0
        stats["entries"] += int(ok.sum())
        stats["ill"] += int((ok & ill).sum())
        for fi, name in enumerate(O.FIELDS):
            a, b = fg[fi, m][ok], fo[fi, m][ok]
            il = ill[ok]
            if name in ("thR",):
                err = np.abs(wrap(a - b))
            elif name in ("thI", "rx", "rz"):
                err = np.abs(a - b)
            elif name == "res":
                assert np.all(a < res_tol) and np.all(b < res_tol)
                continue
            elif name == "Q":
                fin = np.isfinite(b)
                assert np.array_equal(np.isfinite(a), fin)
                err = np.where(fin, np.abs(a - b) / np.where(fin, np.abs(b), 1.0), 0.0)
            else:
                scale = np.abs(b)
                err = np.where(scale > 0, np.abs(a - b) / np.where(scale > 0, scale, 1), np.abs(a - b))
            if err.size:
                stats["max_rel"] = max(stats["max_rel"], float(err[~il].max(initial=0.0)))
                assert np.all(err[~il] <= tol), (name, m, float(err[~il].max()))
                assert np.all(err[il] <= tol_ill), (name, m, "ill")
        # NaN layout of entries without a root
        assert np.all(np.isnan(fg[0, m][blank]))
    return stats


def run_pair(G, classes_np, modes=(0, 1, 2), n_dirs=360, n_sweep=1440, kernel=0):
    import paper_2609_26108_amd as C
    desc = C.cache_desc(n_dirs=n_dirs, modes=modes, kernel=kernel, n_sweep=n_sweep)
    K = classes_np.shape[0]
    cache = G.build_cache(G.classes_from_arrays(classes_np), desc)
    fg, sg = G.cache_to_numpy(cache, desc, K)
    mask = sum(1 << m for m in modes)
    fo, so = O.build_cache_2d(classes_np, n_dirs=n_dirs, mode_mask=mask, reading=kernel,
                              n_sweep=n_sweep)
    return fg, sg, fo, so


def test_cache_rock_table_layers(G, rock_table):
    """All four layers of the paper's rock table, tilted, all three modes
    (layer 1 has a qSV triplication)."""
    cls = []
    for i, r in enumerate(rock_table):
        c = O.class_from_moduli(*(r[:5] * KM2), *r[5:10])
        c[11] = math.radians([0.0, 25.0, -33.0, 71.5][i])
        cls.append(c)
    cls = np.stack(cls)
    fg, sg, fo, so = run_pair(G, cls)
    st = compare_cache(fg, sg, fo, so, (0, 1, 2))
    print("rock table", st)


def test_cache_config1_and_config2_classes(G):
    m1 = W.config1()
    m2 = W.config2()
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m1.layers + m2.layers])
    fg, sg, fo, so = run_pair(G, cls)
    st = compare_cache(fg, sg, fo, so, (0, 1, 2))
    print("config1+2", st)


def test_cache_closed_form_limits(G):
    """Elastic isotropic, elastic VTI, uniform Q and a fluid (no shear)."""
    cls = np.stack([
        O.class_from_thomsen(3000.0, 1732.0, 2300, 0, 0, 0, 0.3, 0, np.inf, np.inf),
        O.class_from_thomsen(3000.0, 1732.0, 2300, 0.2, 0.1, 0.15, 0.0, 0, np.inf, np.inf),
        O.class_from_moduli(14.4e6, 4.5e6, 9.0e6, 2.25e6, 3.0e6, *[50.0] * 5),
        O.class_from_moduli(2.25e6, 2.25e6, 2.25e6, 0.0, 0.0, 1000.0, 1000.0, 1000.0, 1000.0, 1000.0),
    ])
    fg, sg, fo, so = run_pair(G, cls)
    compare_cache(fg, sg, fo, so, (0, 1, 2))
    assert np.all(sg[1, 3] == O.ST_FLUID) and np.all(sg[2, 3] == O.ST_FLUID)
    assert np.all(fg[6, :, 0:2] == 0.0)  # elastic: theta_I exactly 0


def test_cache_small_sizes_and_oev(G, rock_table):
    """Minimum sizes (4 directions, 16 sweep samples) and the OEV kernel on
    qP/qSH (single-root there)."""
    r = rock_table[1]
    c = O.class_from_moduli(*(r[:5] * KM2), *r[5:10])[None]
    fg, sg, fo, so = run_pair(G, c, n_dirs=4, n_sweep=16)
    compare_cache(fg, sg, fo, so, (0, 1, 2))
    fg, sg, fo, so = run_pair(G, c, modes=(0, 2), kernel=1)
    compare_cache(fg, sg, fo, so, (0, 2))


def test_cache_many_random_classes(G):
    """64 random classes across the config-2 parameter ranges (spans many
    workgroups of the solve launch)."""
    rng = np.random.default_rng(99)
    cls = []
    for _ in range(64):
        L = W._layer_params(rng)
        cls.append(O.class_from_thomsen(*L.thomsen_args()))
    cls = np.stack(cls)
    fg, sg, fo, so = run_pair(G, cls, modes=(0, 1))
    st = compare_cache(fg, sg, fo, so, (0, 1))
    print("random64", st)


def test_cache_invalid_class_flags_nonphys(G):
    c = O.class_from_thomsen(3000.0, 1732.0, 2300, 0.2, 0.1, 0.15, 0.0, 0, 60, 40)
    bad = c.copy()
    bad[0] = np.nan
    fg, sg, fo, so = run_pair(G, np.stack([c, bad]), modes=(0,))
    assert np.all(sg[0, 1] == O.ST_NONPHYS)
    assert np.all(np.isnan(fg[0, 0, 1]))


def test_cache_star_subset_columns(G, rock_table):
    """Subset caches (the star's directions only) match the oracle's."""
    import paper_2609_26108_amd as C
    r = rock_table[2]
    cls = np.stack([O.class_from_moduli(*(r[:5] * KM2), *r[5:10], tilt=0.4),
                    O.class_from_thomsen(3000.0, 1732.0, 2300, 0.2, 0.1, 0.15, -0.2, 0, 60, 40)])
    sub = C.star_subset(5, 5.0, 5.0)
    desc = C.cache_desc(modes=(0, 1, 2), subset=sub)
    cache = G.build_cache(G.classes_from_arrays(cls), desc)
    fg, sg = G.cache_to_numpy(cache, desc, 2)
    fo, so = O.build_cache_2d(cls, subset=sub)
    compare_cache(fg, sg, fo, so, (0, 1, 2))


def test_cache_per_node_fused_path(G):
    """One class per node of a small complex model (>= 512 jobs, so the fused
    sweep-in-LDS launch runs), star subset, qSV; classes converted on the
    device (chert_classes_from_thomsen) and by the oracle."""
    import paper_2609_26108_amd as C
    m = W.complex_2d(nx=26, nz=21, h=10.0, water_m=40.0, n_layers=6, n_faults=1, seed=3,
                     radius=3)
    rows = m.param_rows()
    params = torch.from_numpy(rows).to(G.DEV)
    classes = torch.empty((rows.shape[0], 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(params, classes)
    cls_o = np.stack([O.class_from_thomsen(*r) for r in rows])
    torch.cuda.synchronize()
    assert np.array_equal(classes.cpu().numpy(), cls_o)
    sub = C.star_subset(3, m.hx, m.hz)
    desc = C.cache_desc(modes=(1,), n_sweep=720, subset=sub)
    cache = G.build_cache(classes, desc)
    fg, sg = G.cache_to_numpy(cache, desc, rows.shape[0])
    fo, so = O.build_cache_2d(cls_o, mode_mask=0b010, n_sweep=720, subset=sub)
    st = compare_cache(fg, sg, fo, so, (1,))
    print("per-node", st)
