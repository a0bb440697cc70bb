"""Pins of the oracle's slowness-sampled cache (eq 26 read literally: the
cache index is the real slowness angle in the class's symmetry-axis frame)
and of its lookup (the closest stored ray direction by normalised dot
product, text after eq 27) and traveltimes (eqs 28-31)."""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_local import vti_phase_group, wrap


def layer1(rock_table, q=True):
    r = rock_table[0]
    qs = r[5:10] if q else [np.inf] * 5
    return O.class_from_moduli(*(r[:5] * 1e6), *qs)


@pytest.mark.parametrize("tilt", [0.0, 0.4])
def test_isotropic_elastic_samples(tilt):
    """Isotropic elastic: theta_I = 0, V = Vp (Vs), A = 0 and the ray along
    the slowness direction, rotated by the tilt into the global frame."""
    c = O.class_from_thomsen(3000.0, 1700.0, 2300, 0.0, 0.0, 0.0, tilt, 0, np.inf, np.inf)
    n = 360
    f, st = O.build_cache_slow_2d(c, n=n, mode_mask=0b111)
    th = np.arange(n) * 2 * np.pi / n
    for mode, v in ((O.QP, 3000.0), (O.QSV, 1700.0), (O.QSH, 1700.0)):
        assert np.all(st[mode, 0] == 0)
        np.testing.assert_allclose(f[0, mode, 0], v, rtol=1e-14)
        assert np.all(f[1, mode, 0] == 0.0) and np.all(f[6, mode, 0] == 0.0)
        np.testing.assert_allclose(f[3, mode, 0], np.sin(th + tilt), atol=1e-14)
        np.testing.assert_allclose(f[4, mode, 0], np.cos(th + tilt), atol=1e-14)
        np.testing.assert_allclose(f[5, mode, 0], th, atol=0)


@pytest.mark.parametrize("mode", [O.QP, O.QSV])
def test_elastic_vti_closed_form(rock_table, mode):
    """Elastic VTI (layer 1 without Q): at phase angle theta the stored ray
    velocity is the textbook group velocity and the stored direction the
    group angle."""
    c = layer1(rock_table, q=False)
    f, st = O.build_cache_slow_2d(c, n=720, mode_mask=1 << mode)
    th = np.arange(720) * 2 * np.pi / 720
    _, _, Vg, psi = vti_phase_group(c[0], c[1], c[2], c[3], th, qp=(mode == O.QP))
    np.testing.assert_allclose(f[0, mode, 0], Vg, rtol=1e-12)
    np.testing.assert_allclose(wrap(np.arctan2(f[3, mode, 0], f[4, mode, 0]) - psi), 0,
                               atol=1e-12)


def test_uniform_q_direction_is_elastic(rock_table):
    """Uniform Q: Gamma scales by 1 - i/Q, so the eigenvector is real,
    theta_I = 0 and the ray direction is the elastic one."""
    r = rock_table[0]
    c = O.class_from_moduli(*(r[:5] * 1e6), *[40.0] * 5)
    ce = O.class_from_moduli(*(r[:5] * 1e6), *[np.inf] * 5)
    f, _ = O.build_cache_slow_2d(c, n=360, mode_mask=0b011)
    fe, _ = O.build_cache_slow_2d(ce, n=360, mode_mask=0b011)
    for mode in (O.QP, O.QSV):
        assert np.max(np.abs(f[6, mode, 0])) < 1e-12
        np.testing.assert_allclose(f[3, mode, 0], fe[3, mode, 0], atol=1e-11)
        np.testing.assert_allclose(f[4, mode, 0], fe[4, mode, 0], atol=1e-11)


@pytest.mark.parametrize("reading", [O.MEV, O.OEV])
def test_theta_i_is_the_nearest_root(rock_table, reading):
    """Every stored theta_I is the homogeneity root nearest 0 at its theta_R
    (the same definition as the ray-direction cache's inner solve), and the
    residual is at rounding level; layer 1 tilted, every mode."""
    c = layer1(rock_table).copy()
    c[11] = 0.3
    f, st = O.build_cache_slow_2d(c, n=180, mode_mask=0b111, reading=reading)
    for mode in range(3):
        ok = (st[mode, 0] & O.ST_NO_BRACKET) == 0
        assert ok.all()
        for q in range(0, 180, 11):
            assert O.theta_imag(c, mode, f[5, mode, 0, q], reading=reading) == f[6, mode, 0, q]
        assert np.nanmax(f[7, mode, 0]) < 1e-12


def test_fluid_shear_and_layout():
    c = O.class_from_moduli(2.25e6, 2.25e6, 2.25e6, 0.0, 0.0, *[1000.0] * 5)
    f, st = O.build_cache_slow_2d(c, n=36, mode_mask=0b111)
    assert np.all(st[1, 0] == O.ST_FLUID) and np.all(st[2, 0] == O.ST_FLUID)
    assert np.all(np.isnan(f[0, 1, 0]))
    assert np.all(st[0, 0] == 0)


def py_lookup(RX, RZ, st, R, hx, hz):
    offs, L = [], []
    for oz in range(-R, R + 1):
        for ox in range(-R, R + 1):
            if (ox, oz) != (0, 0) and math.gcd(abs(ox), abs(oz)) == 1:
                offs.append((ox, oz))
    K, n = RX.shape
    best = np.full((K, len(offs)), -1, np.int32)
    for o, (ox, oz) in enumerate(offs):
        ex, ez = ox * hx, oz * hz
        ln = math.sqrt(ex * ex + ez * ez)
        dx, dz = ex / ln, ez / ln
        for k in range(K):
            b, bd = -1, 0.0
            for q in range(n):
                if st[k, q] & (O.ST_NO_BRACKET | O.ST_FLUID):
                    continue
                dd = RX[k, q] * dx + RZ[k, q] * dz
                if b < 0 or dd > bd:
                    b, bd = q, dd
            best[k, o] = b
    return offs, best


def random_slow_cache(K, n, rng):
    """Positive V, A and unit ray directions at random angles; some samples
    without a root."""
    ang = rng.uniform(0, 2 * np.pi, (K, n))
    RX, RZ = np.sin(ang), np.cos(ang)
    V = rng.uniform(1500.0, 4500.0, (K, n))
    A = rng.uniform(1e-5, 1e-3, (K, n))
    st = np.zeros((K, n), np.int32)
    st[rng.uniform(size=(K, n)) < 0.1] = O.ST_NO_BRACKET
    return V, A, RX, RZ, st


def test_lookup_is_brute_force_argmax():
    rng = np.random.default_rng(5)
    V, A, RX, RZ, st = random_slow_cache(4, 90, rng)
    for R, hx, hz in ((3, 10.0, 10.0), (5, 5.0, 7.5)):
        _, ref = py_lookup(RX, RZ, st, R, hx, hz)
        np.testing.assert_array_equal(O.slow_lookup(RX, RZ, st, R, hx, hz), ref)


def test_trace_equals_bellman_ford():
    """Dijkstra on a slowness-sampled cache equals Bellman-Ford sweeps with
    the per-endpoint lookup and eqs 28-30 evaluated in Python, bitwise, for
    both fields on a small grid with three classes."""
    rng = np.random.default_rng(8)
    K, n, R = 3, 72, 2
    V, A, RX, RZ, st = random_slow_cache(K, n, rng)
    nx, nz, hx, hz = 7, 6, 10.0, 8.0
    cid = rng.integers(0, K, nx * nz).astype(np.int32)
    offs, best = py_lookup(RX, RZ, st, R, hx, hz)
    f = np.zeros((O.NF, K, n))
    f[0], f[1], f[3], f[4] = V, A, RX, RZ
    src = 9
    o = O.trace_2d_slow(nx, nz, hx, hz, cid, R, f, st, src)
    for field, key in ((0, "tauR"), (1, "tauI")):
        tau = np.full(nx * nz, np.inf)
        tau[src] = 0.0
        for _ in range(nx * nz):
            for i in range(nx * nz):
                if not np.isfinite(tau[i]):
                    continue
                ix, iz = i % nx, i // nx
                for oo, (ox, oz) in enumerate(offs):
                    jx, jz = ix + ox, iz + oz
                    if not (0 <= jx < nx and 0 <= jz < nz):
                        continue
                    j = jx + nx * jz
                    ci, cj = best[cid[i], oo], best[cid[j], oo]
                    L = math.sqrt((ox * hx) ** 2 + (oz * hz) ** 2)
                    if ci < 0 or cj < 0 or st[cid[i], ci] or st[cid[j], cj]:
                        continue
                    if field == 0:
                        w = L / (0.5 * (V[cid[i], ci] + V[cid[j], cj]))
                    else:
                        w = L * (0.5 * (A[cid[i], ci] + A[cid[j], cj]))
                    if tau[i] + w < tau[j]:
                        tau[j] = tau[i] + w
        np.testing.assert_array_equal(o[key], tau)


def test_isotropic_field_matches_ray_direction_cache():
    """Isotropic elastic medium with an integer-degree tilt: each edge's
    closest stored ray direction is its own 1-degree bin, so the traveltimes
    equal those through the ray-direction cache (to rounding in V)."""
    c = O.class_from_thomsen(3000.0, 1700.0, 2300, 0.0, 0.0, 0.0, math.radians(20), 0,
                             np.inf, np.inf)
    nx, nz, R = 41, 31, 4
    cid = np.zeros(nx * nz, np.int32)
    fs, ss = O.build_cache_slow_2d(c, n=360, mode_mask=0b001)
    fr, sr = O.build_cache_2d(c, n_dirs=360, mode_mask=0b001, n_sweep=720)
    a = O.trace_2d_slow(nx, nz, 10.0, 10.0, cid, R, fs[:, 0], ss[0], 600)
    b = O.trace_2d(nx, nz, 10.0, 10.0, cid, R, fr[0, 0], fr[1, 0], sr[0], 600)
    # (predecessors are not compared: a homogeneous medium has many paths of
    # equal length, and V differing in the last bits re-decides those ties)
    np.testing.assert_allclose(a["tauR"], b["tauR"], rtol=1e-13)
