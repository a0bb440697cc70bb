"""Pins of the oracle's 3D part: Fibonacci directions, the 3D star, the
sagittal-plane cache (checked by an independent 3x3 complex Christoffel
solve with the stiffness rotated by eq 35), and 3D Dijkstra (brute force,
straight-ray gauge, predecessor folds)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

KM2 = 1e6


def test_fibonacci_directions():
    f = O.fibonacci()
    assert f.shape == (O.N_FIB, 3)
    np.testing.assert_allclose(np.linalg.norm(f, axis=1), 1.0, atol=3e-16)
    assert np.abs(f.mean(0)).max() < 1e-6
    # nearest-neighbour spacing of a sample: about one degree
    rng = np.random.default_rng(0)
    pick = rng.choice(O.N_FIB, 300, replace=False)
    d = f[pick] @ f.T
    d[np.arange(300), pick] = -2.0
    nn = np.degrees(np.arccos(np.clip(d.max(1), -1, 1)))
    assert 0.8 < nn.min() and nn.max() < 1.05


def test_star_3d_definition():
    """|O_3| = 290 by brute force; (oy, oz, ox) order; lengths are norms;
    bins maximise the dot product (numpy argmax, first on ties); distinct;
    the oy = 0 offsets are the 2D star in its order."""
    R, hx, hy, hz = 3, 10.0, 12.0, 8.0
    ox, oy, oz, L, b = O.star_3d(R, hx, hy, hz)
    ref = [(y, z, x) for y in range(-R, R + 1) for z in range(-R, R + 1)
           for x in range(-R, R + 1)
           if (x, y, z) != (0, 0, 0) and math.gcd(math.gcd(abs(x), abs(y)), abs(z)) == 1]
    assert len(ref) == 290 == len(ox)
    assert [(y, z, x) for x, y, z in zip(ox, oy, oz)] == ref
    v = np.stack([ox * hx, oy * hy, oz * hz], 1)
    np.testing.assert_allclose(L, np.linalg.norm(v, axis=1), rtol=2e-16)
    f = O.fibonacci()
    u = v / np.linalg.norm(v, axis=1)[:, None]
    assert np.array_equal(b, np.argmax(u @ f.T, axis=1))
    assert len(set(b.tolist())) == 290
    ox2, oz2, _, _ = O.star_2d(R, hx, hz)
    sel = oy == 0
    assert np.array_equal(ox[sel], ox2) and np.array_equal(oz[sel], oz2)


# ---------------------------------------------------------------------------
# independent 3D check of the sagittal reduction

def voigt_ti(c):
    """Complex 6x6 Voigt stiffness of a TI class in its axis frame (eq 2)."""
    def m(a, q):
        return a * (1 - 1j / q) if np.isfinite(q) else complex(a)
    a11, a13, a33, a44, a66 = (m(c[i], c[5 + i]) for i in range(5))
    C = np.zeros((6, 6), complex)
    C[0, 0] = C[1, 1] = a11
    C[2, 2] = a33
    C[0, 1] = C[1, 0] = a11 - 2 * a66
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = a13
    C[3, 3] = C[4, 4] = a44
    C[5, 5] = a66
    return C


VOIGT = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3, (0, 2): 4, (2, 0): 4,
         (0, 1): 5, (1, 0): 5}


def tensor(C):
    c = np.zeros((3, 3, 3, 3), complex)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    c[i, j, k, l] = C[VOIGT[i, j], VOIGT[k, l]]
    return c


def basis_eq35(t0, p0):
    ex = np.array([math.cos(t0) * math.cos(p0), math.cos(t0) * math.sin(p0), -math.sin(t0)])
    ey = np.array([-math.sin(p0), math.cos(p0), 0.0])
    ez = np.array([math.sin(t0) * math.cos(p0), math.sin(t0) * math.sin(p0), math.cos(t0)])
    return np.stack([ex, ey, ez])  # rows: local axes in global coordinates


def global_energy_velocity(cls, mode, n):
    """3x3 complex Christoffel solve (eq 4) with the rotated tensor, MEV
    energy velocity v_m = c_mjkl p_l Re(g_j g_k*)/(g^H g)."""
    Rm = basis_eq35(cls[11], cls[12])
    c = np.einsum("ai,bj,ck,dl,abcd->ijkl", Rm, Rm, Rm, Rm, tensor(voigt_ti(cls)))
    G = np.einsum("ijkl,i,l->jk", c, n, n)
    ev, vec = np.linalg.eig(G)
    # mode selection: qSH polarised off the sagittal plane, qP the largest
    # remaining Re G
    ez = Rm[2]
    ysag = np.cross(ez, n.real)
    ysag /= np.linalg.norm(ysag)
    sh = int(np.argmax(np.abs(ysag @ vec)))
    rest = [q for q in range(3) if q != sh]
    if mode == 2:
        q = sh
    else:
        q = max(rest, key=lambda r: ev[r].real) if mode == 0 else min(rest, key=lambda r: ev[r].real)
    g = vec[:, q]
    cc = np.sqrt(ev[q])
    if cc.real < 0:
        cc = -cc
    p = n / cc
    S = np.real(np.outer(g, g.conj())) / np.real(g.conj() @ g)
    return np.einsum("mjkl,l,jk->m", c, p, S)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_sagittal_cache_solves_the_3d_problem(rock_table, mode):
    """For tilted and azimuthally rotated classes, entry i's (theta_R,
    theta_I), placed in the plane of the axis and f_i, solves the full 3D
    problem: v^R and v^I both along f_i (homogeneous, ray direction f_i),
    and V, A of eq 11 equal the cached ones."""
    r = rock_table[1]
    classes = [O.class_from_moduli(*(r[:5] * KM2), *r[5:10], tilt=0.6, azimuth=1.1),
               O.class_from_thomsen(3000.0, 1732.0, 2300, 0.2, 0.1, 0.15, -0.4, 2.5, 60, 40)]
    N = 2000
    f, s = O.build_cache_3d(np.stack(classes), N=N, mode_mask=1 << mode, n_sweep=720)
    fib = O.fibonacci(N)
    rng = np.random.default_rng(mode)
    for k, cls in enumerate(classes):
        ez = basis_eq35(cls[11], cls[12])[2]
        for i in rng.choice(N, 25, replace=False):
            if s[mode, k, i] != 0:
                continue
            fi = fib[i]
            xs = fi - (fi @ ez) * ez
            xs /= np.linalg.norm(xs)
            z = f[5, mode, k, i] + 1j * f[6, mode, k, i]
            n = np.sin(z) * xs + np.cos(z) * ez
            v = global_energy_velocity(cls, mode, n)
            vR, vI = v.real, v.imag
            assert np.linalg.norm(vR / np.linalg.norm(vR) - fi) < 1e-9
            if np.linalg.norm(vI) > 0:
                assert np.linalg.norm(vI - (vI @ fi) * fi) <= 1e-8 * np.linalg.norm(vI)
            vr = np.linalg.norm(vR)
            vi = vI @ fi
            np.testing.assert_allclose(f[0, mode, k, i], (vr ** 2 + vi ** 2) / vr, rtol=1e-9)
            np.testing.assert_allclose(f[1, mode, k, i], -vi / (vr ** 2 + vi ** 2), rtol=1e-8)
            assert f[3, mode, k, i] == fi[0] and f[4, mode, k, i] == fi[2]


def test_isotropic_elastic_3d_is_uniform():
    c = O.class_from_thomsen(3000.0, 1732.0, 2300, 0, 0, 0, 0.3, 1.0, np.inf, np.inf)
    f, s = O.build_cache_3d(c, N=500, mode_mask=0b111, n_sweep=360)
    np.testing.assert_allclose(f[0, 0, 0], 3000.0, rtol=1e-13)
    np.testing.assert_allclose(f[0, 1, 0], 1732.0, rtol=1e-13)
    np.testing.assert_allclose(f[0, 2, 0], 1732.0, rtol=1e-13)
    assert np.all(f[1] [:, 0] == 0.0)


# ---------------------------------------------------------------------------
# 3D graph

def _small_3d(seed, nx=6, ny=5, nz=4, R=2, N=800, mode=1):
    rng = np.random.default_rng(seed)
    layers = [W._layer_params(rng) for _ in range(2)]
    cls = []
    for L in layers:
        c = O.class_from_thomsen(*L.thomsen_args())
        c[12] = rng.uniform(0, 2 * np.pi)
        cls.append(c)
    cls = np.stack(cls)
    f, s = O.build_cache_3d(cls, N=N, mode_mask=1 << mode, n_sweep=360)
    cid = (rng.random((nz, ny, nx)) < 0.5).astype(np.int32)
    return cls, f, s, cid


def _bellman_ford(nx, ny, nz, hx, hy, hz, cid, R, N, V, A, st, src, field):
    ox, oy, oz, L, b = O.star_3d(R, hx, hy, hz, N)
    n = nx * ny * nz
    tau = np.full(n, np.inf)
    tau[src] = 0.0
    bad = 1 | 4 | 8
    ok = (st & bad) == 0
    changed = True
    while changed:
        changed = False
        for i in range(n):
            if not np.isfinite(tau[i]):
                continue
            x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
            for o in range(len(ox)):
                X, Y, Z = x + ox[o], y + oy[o], z + oz[o]
                if not (0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz):
                    continue
                j = X + nx * (Y + ny * Z)
                ki, kj, c = cid.flat[i], cid.flat[j], b[o]
                if not (ok[ki, c] and ok[kj, c]):
                    continue
                if field == 0:
                    w = L[o] / (0.5 * (V[ki, c] + V[kj, c]))
                else:
                    w = L[o] * (0.5 * (A[ki, c] + A[kj, c]))
                cand = tau[i] + w
                if cand < tau[j]:
                    tau[j] = cand
                    changed = True
    return tau


@pytest.mark.parametrize("R", [1, 2])
def test_dijkstra_3d_equals_brute_force(R):
    cls, f, s, cid = _small_3d(3, R=R)
    nx, ny, nz = 6, 5, 4
    src = 2 + nx * (1 + ny * 1)
    o = O.trace_3d(nx, ny, nz, 10.0, 10.0, 10.0, cid, R, f[0, 1], f[1, 1], s[1], src, N=800)
    for field, key in ((0, "tauR"), (1, "tauI")):
        bf = _bellman_ford(nx, ny, nz, 10.0, 10.0, 10.0, cid, R, 800, f[0, 1], f[1, 1], s[1],
                           src, field)
        assert np.array_equal(o[key], bf), key


def test_pred_3d_folds_to_tau():
    cls, f, s, cid = _small_3d(4, nx=7, ny=6, nz=5, R=2)
    nx, ny, nz = 7, 6, 5
    src = 0
    o = O.trace_3d(nx, ny, nz, 10.0, 10.0, 10.0, cid, 2, f[0, 1], f[1, 1], s[1], src, N=800)
    ox, oy, oz, L, b = O.star_3d(2, 10.0, 10.0, 10.0, 800)
    V = f[0, 1]
    for j in range(1, nx * ny * nz):
        if not np.isfinite(o["tauR"][j]):
            assert o["predP"][j] == -1
            continue
        path = [j]
        while path[-1] != src:
            path.append(int(o["predP"][path[-1]]))
            assert len(path) <= nx * ny * nz
        t = 0.0
        for a, c in zip(path[::-1][:-1], path[::-1][1:]):
            d = (c % nx - a % nx, (c // nx) % ny - (a // nx) % ny, c // (nx * ny) - a // (nx * ny))
            oo = [q for q in range(len(ox)) if (ox[q], oy[q], oz[q]) == d][0]
            ki, kj = cid.flat[a], cid.flat[c]
            t = t + L[oo] / (0.5 * (V[ki, b[oo]] + V[kj, b[oo]]))
        assert t == o["tauR"][j]


def test_homogeneous_isotropic_straight_rays_3d():
    """Along every star direction from the source the traveltime is the
    fold of k equal weights L/V: straight rays (graph gauge)."""
    c = O.class_from_thomsen(3000.0, 1732.0, 2300, 0, 0, 0, 0.0, 0.0, np.inf, np.inf)
    N = 800
    f, s = O.build_cache_3d(c, N=N, mode_mask=1, n_sweep=360)
    nx = ny = nz = 7
    cid = np.zeros((nz, ny, nx), np.int32)
    src = 3 + nx * (3 + ny * 3)
    o = O.trace_3d(nx, ny, nz, 10.0, 10.0, 10.0, cid, 1, f[0, 0], f[1, 0], s[0], src, N=N)
    ox, oy, oz, L, b = O.star_3d(1, 10.0, 10.0, 10.0, N)
    for q in range(len(ox)):
        t = 0.0
        for k in range(1, 4):
            t = t + L[q] / 3000.0
            j = (3 + k * ox[q]) + nx * ((3 + k * oy[q]) + ny * (3 + k * oz[q]))
            assert o["tauR"][j] == t


def test_tstar_3d_is_the_fold_along_pred():
    """t* of every reached node is the left-to-right fold of the attenuation
    weights along its propagation raypath (eq 30 on the pred_P tree)."""
    cls, f, s, cid = _small_3d(6, nx=6, ny=5, nz=4, R=2)
    nx, ny, nz = 6, 5, 4
    src = 7
    o = O.trace_3d(nx, ny, nz, 10.0, 10.0, 10.0, cid, 2, f[0, 1], f[1, 1], s[1], src, N=800)
    ox, oy, oz, L, b = O.star_3d(2, 10.0, 10.0, 10.0, 800)
    A = f[1, 1]
    for j in range(nx * ny * nz):
        if not np.isfinite(o["tauR"][j]):
            assert o["tstar"][j] == np.inf
            continue
        path = [j]
        while path[-1] != src:
            path.append(int(o["predP"][path[-1]]))
        t = 0.0
        for a, c in zip(path[::-1][:-1], path[::-1][1:]):
            d = (c % nx - a % nx, (c // nx) % ny - (a // nx) % ny, c // (nx * ny) - a // (nx * ny))
            q = [k for k in range(len(ox)) if (ox[k], oy[k], oz[k]) == d][0]
            t = t + L[q] * (0.5 * (A[cid.flat[a], b[q]] + A[cid.flat[c], b[q]]))
        assert t == o["tstar"][j]
