"""Pins of the surrogate oracle (oracle/surrogate.py) against things other
than itself: a library rounding routine, a library optimiser, finite
differences, closed-form networks and closed-form cache entries."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import surrogate as S

torch = pytest.importorskip("torch")


def _rand_params(rng, scale=0.3):
    return rng.normal(0.0, scale, S.N_PARAMS)


def test_bf16_matches_library_rounding():
    """Round-to-nearest-even float32 -> bfloat16 equals torch's conversion,
    including ties, subnormals, infinities and signed zeros."""
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.normal(0, 1, 20000).astype(np.float32),
        (rng.normal(0, 1, 2000) * 1e-39).astype(np.float32),       # subnormal
        np.array([0.0, -0.0, np.inf, -np.inf, 1.0, 3.0e38], np.float32),
        # exact ties: low 16 bits 0x8000 with even and odd kept parts
        np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x00018000],
                 np.uint32).view(np.float32),
    ])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = S.bf16(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(S.bf16(np.array([np.nan], np.float32))[0])


def test_single_path_network_closed_form():
    """Only W1[2][5], W2[5][7], W3[7][1], W4[1][3] and b4 nonzero: output 3
    is d tanh(c tanh(b tanh(a x_2))) + b4[3], the others are b4.  A
    transposed weight or a swapped layer order breaks it."""
    w = {name: np.zeros(shp) for name, shp in S.SHAPES}
    a, b, c, d = 0.7, -1.3, 0.9, 2.5
    w["W1"][2, 5] = a
    w["W2"][5, 7] = b
    w["W3"][7, 1] = c
    w["W4"][1, 3] = d
    w["b4"][:] = [0.1, -0.2, 0.3, 0.4]
    p = S.pack(w)
    X = np.random.default_rng(2).normal(0, 1, (9, S.N_IN))
    out, _ = S.forward(p, X)
    for i in range(9):
        exp = d * math.tanh(c * math.tanh(b * math.tanh(a * X[i, 2]))) + 0.4
        assert abs(out[i, 3] - exp) < 1e-15
        assert np.all(out[i, :3] == w["b4"][:3])


def test_biases_only_network():
    """Zero weights: every hidden unit is tanh of its bias; the output is
    tanh(b3) @ W4 + b4 whatever the input."""
    rng = np.random.default_rng(3)
    w = {name: np.zeros(shp) for name, shp in S.SHAPES}
    for name in ("b1", "b2", "b3", "b4", "W4"):
        w[name] = rng.normal(0, 1, w[name].shape)
    out, _ = S.forward(S.pack(w), rng.normal(0, 1, (4, S.N_IN)))
    exp = np.tanh(w["b3"]) @ w["W4"] + w["b4"]
    np.testing.assert_allclose(out, np.broadcast_to(exp, out.shape), rtol=1e-14)


def test_gradient_matches_central_differences():
    """Backward (FP64) against central differences of the loss on 74
    coordinates spread over all eight parameter blocks (b4 has 4): 1e-7 relative."""
    rng = np.random.default_rng(4)
    p = _rand_params(rng)
    X = rng.normal(0, 1, (12, S.N_IN))
    Y = rng.normal(0, 1, (12, S.N_OUT))
    L, g = S.backward(p, X, Y)
    assert abs(L - S.loss(p, X, Y)) < 1e-15
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in S.SHAPES])
    idx = np.concatenate([rng.choice(np.arange(offs[i], offs[i + 1]),
                                     min(10, offs[i + 1] - offs[i]), replace=False)
                          for i in range(8)])
    gmax = np.abs(g).max()
    h = 1e-5
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (S.loss(p + e, X, Y) - S.loss(p - e, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-3 * gmax), (i, fd, g[i])


def test_adam_matches_library_optimiser():
    """Three Adam steps against torch.optim.Adam (CPU, FP64) with the same
    gradients, betas and epsilon."""
    rng = np.random.default_rng(5)
    p0 = rng.normal(0, 1, 50)
    grads = [rng.normal(0, 1, 50) * 10.0 ** k for k in (0, -2, 1)]
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(S.BETA1, S.BETA2), eps=S.ADAM_EPS)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = S.adam(p, m, v, g, t, 3e-3)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-14, atol=1e-16)


def test_bf16_forms_track_fp64():
    """The device-precision forward and gradient stay within BF16 accuracy
    of the FP64 ones (forward 2e-2 of the output range, gradient cosine
    similarity > 0.999)."""
    rng = np.random.default_rng(6)
    p = _rand_params(rng, 0.1)
    X = rng.normal(0, 1, (64, S.N_IN))
    Y = rng.normal(0, 1, (64, S.N_OUT))
    o64, _ = S.forward(p, X)
    o16, _ = S.forward_bf16(p.astype(np.float32), X.astype(np.float32))
    assert np.abs(o16 - o64).max() < 2e-2 * np.abs(o64).max()
    _, g64 = S.backward(p, X, Y)
    _, g16 = S.backward_bf16(p.astype(np.float32), X.astype(np.float32), Y.astype(np.float32))
    cos = float(g64 @ g16 / (np.linalg.norm(g64) * np.linalg.norm(g16)))
    assert cos > 0.999, cos


def test_features_of_a_thomsen_class():
    """a11/a33 - 1 = 2 eps, a44/a33 = (Vs0/Vp0)^2, a66/a33 = that times
    (1 + 2 gamma) (Thomsen 1986), inverse Q per modulus, mode one-hot, the
    angle's harmonics; an elastic class has zero inverse Q."""
    c = O.class_from_thomsen(3000.0, 1500.0, 2300, 0.2, 0.1, 0.15, 0.3, 0, 60, 40)
    f = S.features(c, 1, 0.25)
    assert abs(f[0] - 0.4) < 1e-15
    assert abs(f[2] - 0.25) < 1e-15
    assert abs(f[3] - 0.25 * 1.3) < 1e-15
    np.testing.assert_allclose(f[4:9], [1 / 60, 1 / 60, 1 / 60, 1 / 40, 1 / 40], rtol=1e-15)
    assert list(f[9:12]) == [0.0, 1.0, 0.0]
    np.testing.assert_allclose(f[12:], [math.cos(0.25), math.sin(0.25), math.cos(0.5),
                                        math.sin(0.5)], rtol=1e-15)
    ce = O.class_from_thomsen(3000.0, 1500.0, 2300, 0.2, 0.1, 0.15, 0.3, 0, np.inf, np.inf)
    assert np.all(S.features(ce, 0, 0.0)[4:9] == 0.0)


def test_targets_of_isotropic_caches():
    """Isotropic elastic: theta_R = psi, theta_I = 0, V = sqrt(a) of the
    mode, A = 0.  Isotropic viscoelastic: V = |c|^2/Re c and
    A = -Im c/|c|^2 with c = sqrt(a (1 - i/Q)) (eqs 2, 11)."""
    M, mu = 9.0e6, 2.0e6
    ce = O.class_from_moduli(M, M - 2 * mu, M, mu, mu, *[np.inf] * 5, tilt=0.4)
    f, st = O.build_cache_2d(ce, n_dirs=24)
    X, Y, ok = S.dataset_from_cache(ce[None], f, st, n_dirs=24)
    assert ok.all()
    Y = Y.reshape(3, 24, 4)
    assert np.abs(Y[..., 0]).max() < 1e-12 and np.all(Y[..., 1] == 0.0)
    np.testing.assert_allclose(Y[0, :, 2], 0.0, atol=1e-14)
    np.testing.assert_allclose(Y[1:, :, 2], 0.5 * math.log(mu / M), rtol=1e-13)
    assert np.all(Y[..., 3] == 0.0)
    # local angle of column d is d*15 deg - tilt, wrapped
    psi = np.arctan2(X[:24, 13], X[:24, 12])
    d = np.arange(24) * (2 * np.pi / 24) - 0.4
    np.testing.assert_allclose(np.angle(np.exp(1j * (psi - d))), 0.0, atol=1e-14)

    Qp, Qs = 60.0, 40.0
    a13I = M / Qp - 2 * mu / Qs
    cq = O.class_from_moduli(M, M - 2 * mu, M, mu, mu, Qp, (M - 2 * mu) / a13I, Qp, Qs, Qs)
    f, st = O.build_cache_2d(cq, n_dirs=8)
    _, Y, ok = S.dataset_from_cache(cq[None], f, st, n_dirs=8)
    Y = Y.reshape(3, 8, 4)
    for mode, (a, Q) in [(0, (M, Qp)), (1, (mu, Qs)), (2, (mu, Qs))]:
        cc = np.sqrt(a * (1 - 1j / Q))
        np.testing.assert_allclose(Y[mode, :, 2], math.log(abs(cc) ** 2 / cc.real / math.sqrt(M)),
                                   rtol=1e-12)
        np.testing.assert_allclose(Y[mode, :, 3], -cc.imag / abs(cc) ** 2 * math.sqrt(M),
                                   rtol=1e-11)


def test_standardisation_invariants():
    rng = np.random.default_rng(7)
    X = rng.normal(3, 2, (500, S.N_IN))
    X[:, 9] = 1.0  # constant column: scale taken as 1
    Y = rng.normal(-1, 0.1, (500, S.N_OUT))
    ok = rng.random(500) < 0.7
    mx, sx, my, sy = S.norm_stats(X, Y, ok)
    Xs = (X[ok] - mx) / sx
    np.testing.assert_allclose(Xs.mean(0), 0.0, atol=1e-12)
    np.testing.assert_allclose(np.delete(Xs.std(0), 9), 1.0, rtol=1e-12)
    assert sx[9] == 1.0 and np.all(Xs[:, 9] == 0.0)
    np.testing.assert_allclose(((Y[ok] - my) / sy).std(0), 1.0, rtol=1e-12)


def test_fp64_training_reduces_loss():
    """A few hundred full-batch Adam steps fit a smooth 2-output function of
    the inputs: the loss falls by 10x (the pieces compose into training)."""
    rng = np.random.default_rng(8)
    X = rng.normal(0, 1, (256, S.N_IN))
    Y = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 12], X[:, 1] * X[:, 2], 0.3 * X[:, 5],
                  np.cos(X[:, 13])], axis=1)
    lim = np.sqrt(6.0 / (S.N_IN + S.HID))
    p = S.pack({name: (rng.uniform(-lim, lim, shp) if name[0] == "W" else np.zeros(shp))
                for name, shp in S.SHAPES})
    m, v = np.zeros_like(p), np.zeros_like(p)
    L0 = S.loss(p, X, Y)
    for t in range(1, 301):
        _, g = S.backward(p, X, Y)
        p, m, v = S.adam(p, m, v, g, t, 3e-3)
    assert S.loss(p, X, Y) < 0.1 * L0
