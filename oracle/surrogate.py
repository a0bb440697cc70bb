"""Surrogate oracle -- test infrastructure only (tests, smoke, CPU baseline).

A plain numpy reference of the learned surrogate that warm-starts the cache
solve.  The surrogate is not part of the paper's method: the paper finds that
grouping a structurally complex model into a few property classes is too
coarse and that a per-node cache would be needed (application to the
Marmousi-type model; conclusions), and the surrogate is the device that makes
per-node caches affordable.  The plain solver stays its judge: every warm
started entry is polished on the homogeneity/direction equations (eq 9 and
the target ray direction of eq 26) and checked before it is kept.

What is defined here, in FP64 unless stated:
  features(class, mode, psi_local)   16 inputs, dimensionless
  targets(entry)                      4 outputs per cache entry
  forward / backward                  MLP 16 -> 128 -> 128 -> 128 -> 4, tanh
                                      hidden layers, linear output, MSE loss
  adam                                the Adam update (Kingma and Ba, 2015)
  forward_bf16 / backward_bf16        the same with the device's precision
                                      choices: BF16 operands of every matrix
                                      product, FP32 accumulation, FP32 bias,
                                      tanh and loss; activations kept in BF16
                                      (the tanh derivative uses them).

Parameter vector (FP32 master copy, this order): W1[16][128], b1[128],
W2[128][128], b2[128], W3[128][128], b3[128], W4[128][4], b4[4]; a layer maps
x -> x @ W + b.
"""
from __future__ import annotations

import numpy as np

N_IN, HID, N_OUT = 16, 128, 4
SHAPES = [("W1", (N_IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, N_OUT)), ("b4", (N_OUT,))]
N_PARAMS = int(sum(np.prod(s) for _, s in SHAPES))
FEATURES = ("a11/a33-1", "a13/a33", "a44/a33", "a66/a33", "1/q11", "1/q13", "1/q33",
            "1/q44", "1/q66", "qP", "qSV", "qSH", "cos psi", "sin psi", "cos 2psi",
            "sin 2psi")
TARGETS = ("thR-psi", "thI", "log V/sqrt(a33)", "A sqrt(a33)")


def unpack(p):
    """Flat parameter vector -> dict of views."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d, dtype=np.float64):
    return np.concatenate([np.asarray(d[name], dtype=dtype).reshape(-1) for name, _ in SHAPES])


# ------------------------------------------------------------ data ---------

def _inv_q(q):
    q = np.asarray(q, dtype=np.float64)
    return np.where(np.isinf(q), 0.0, 1.0 / np.where(np.isinf(q), 1.0, q))


def features(cls, mode, psi_local):
    """Inputs of one or many samples.  cls: [..., 13] class rows (moduli,
    Q per modulus, rho, tilt, azimuth); mode 0/1/2; psi_local: target ray
    angle in the symmetry-axis frame (eq 36).  The kinematics of a TI medium
    depend on the moduli only through their ratios (a common factor scales
    every velocity by its square root), so the inputs are the ratios to a33,
    the inverse quality factors (eq 2), the mode and the angle."""
    cls = np.asarray(cls, dtype=np.float64)
    psi = np.asarray(psi_local, dtype=np.float64)
    mode = np.asarray(mode)
    shape = np.broadcast_shapes(cls.shape[:-1], psi.shape, mode.shape)
    cls = np.broadcast_to(cls, shape + (13,))
    psi = np.broadcast_to(psi, shape)
    mode = np.broadcast_to(mode, shape)
    a11, a13, a33, a44, a66 = (cls[..., i] for i in range(5))
    f = np.zeros(shape + (N_IN,))
    f[..., 0] = a11 / a33 - 1.0
    f[..., 1] = a13 / a33
    f[..., 2] = a44 / a33
    f[..., 3] = a66 / a33
    for i in range(5):
        f[..., 4 + i] = _inv_q(cls[..., 5 + i])
    for m in range(3):
        f[..., 9 + m] = (mode == m).astype(np.float64)
    f[..., 12] = np.cos(psi)
    f[..., 13] = np.sin(psi)
    f[..., 14] = np.cos(2.0 * psi)
    f[..., 15] = np.sin(2.0 * psi)
    return f


def _wrap(a):
    return np.where(a > np.pi, a - 2 * np.pi, np.where(a <= -np.pi, a + 2 * np.pi, a))


def targets(cls, psi_local, thR, thI, V, A):
    """Outputs of a cache entry: slowness angle relative to the target ray
    angle, theta_I, log of V over sqrt(a33), A times sqrt(a33) (eqs 9-11;
    the last two are scale free like the inputs)."""
    cls = np.asarray(cls, dtype=np.float64)
    s = np.sqrt(cls[..., 2])
    y = np.stack([_wrap(np.asarray(thR) - np.asarray(psi_local)), np.asarray(thI),
                  np.log(np.asarray(V) / s), np.asarray(A) * s], axis=-1)
    return y


def dataset_from_cache(classes, fields, status, n_dirs=360, subset=None, modes=(0, 1, 2)):
    """(X [n][16], Y [n][4], ok [n]) over every (mode, class, column) of a
    cache in that order; ok marks entries with status OK (the only ones
    used for training)."""
    classes = np.atleast_2d(np.asarray(classes, dtype=np.float64))
    K = classes.shape[0]
    cols = np.arange(n_dirs) if subset is None else np.asarray(subset)
    psi_g = cols * (2 * np.pi / n_dirs)
    Xs, Ys, oks = [], [], []
    for m in modes:
        psi = _wrap(psi_g[None, :] - classes[:, 11:12])          # [K][n_cols]
        X = features(classes[:, None, :], np.full(psi.shape, m), psi)
        Y = targets(classes[:, None, :], psi, fields[5, m], fields[6, m],
                    fields[0, m], fields[1, m])
        ok = status[m] == 0
        Xs.append(X.reshape(-1, N_IN))
        Ys.append(Y.reshape(-1, N_OUT))
        oks.append(ok.reshape(-1))
    return np.concatenate(Xs), np.concatenate(Ys), np.concatenate(oks)


def norm_stats(X, Y, ok):
    """Per-column shift and scale of the standardisation, over the OK
    samples: x_s = (x - mean) / std, a zero std taken as 1."""
    Xo, Yo = np.asarray(X, np.float64)[ok], np.asarray(Y, np.float64)[ok]
    mx, sx = Xo.mean(0), Xo.std(0)
    my, sy = Yo.mean(0), Yo.std(0)
    sx = np.where(sx > 0, sx, 1.0)
    sy = np.where(sy > 0, sy, 1.0)
    return mx, sx, my, sy


# ------------------------------------------------------------ MLP FP64 -----

def forward(p, Xs):
    """Returns (out, activations [x, h1, h2, h3])."""
    w = unpack(np.asarray(p, dtype=np.float64))
    h = [np.asarray(Xs, dtype=np.float64)]
    for l in (1, 2, 3):
        h.append(np.tanh(h[-1] @ w[f"W{l}"] + w[f"b{l}"]))
    out = h[-1] @ w["W4"] + w["b4"]
    return out, h


def loss(p, Xs, Ys):
    """Mean of the squared error over samples and outputs."""
    out, _ = forward(p, Xs)
    return float(np.mean((out - Ys) ** 2))


def backward(p, Xs, Ys):
    """(loss, gradient of the loss as a flat vector), by the chain rule."""
    w = unpack(np.asarray(p, dtype=np.float64))
    out, h = forward(p, Xs)
    B = Xs.shape[0]
    d = 2.0 * (out - Ys) / (B * N_OUT)
    g = {"W4": h[3].T @ d, "b4": d.sum(0)}
    dh = d @ w["W4"].T
    for l in (3, 2, 1):
        dz = dh * (1.0 - h[l] ** 2)
        g[f"W{l}"] = h[l - 1].T @ dz
        g[f"b{l}"] = dz.sum(0)
        dh = dz @ w[f"W{l}"].T
    return float(np.mean((out - Ys) ** 2)), pack(g)


# ------------------------------------------------------------ Adam ---------

BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam(p, m, v, g, t, lr):
    """One Adam step (t counts from 1), bias-corrected moments; returns new
    (p, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** t)
    vh = v / (1.0 - BETA2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


# ------------------------------------------------------------ BF16 ---------

def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32: keep the top 16 bits after adding half an ulp of the kept
    part plus the tie-breaking bit."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(a), (u | 0x400000) & 0xFFFF0000, r)
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def _mm(a, b):
    """BF16 operands, FP32 result (accumulated in FP64 and rounded once;
    the device accumulates in FP32 in its own order)."""
    return (bf16(a).astype(np.float64) @ bf16(b).astype(np.float64)).astype(np.float32)


def forward_bf16(p, Xs):
    """Device-precision forward: returns (out fp32, [x, h1, h2, h3] as the
    BF16 values the device keeps)."""
    w = unpack(np.asarray(p, dtype=np.float32))
    h = [bf16(Xs)]
    for l in (1, 2, 3):
        z = _mm(h[-1], w[f"W{l}"]) + w[f"b{l}"].astype(np.float32)
        h.append(bf16(np.tanh(z.astype(np.float32))))
    out = _mm(h[-1], w["W4"]) + w["b4"].astype(np.float32)
    return out.astype(np.float32), h


def backward_bf16(p, Xs, Ys):
    """Device-precision gradient: the output error and every back-propagated
    error are rounded to BF16 before they enter a product; bias gradients
    sum the BF16 errors in FP32; the tanh derivative uses the BF16
    activations."""
    w = unpack(np.asarray(p, dtype=np.float32))
    out, h = forward_bf16(p, Xs)
    B = Xs.shape[0]
    e = out - np.asarray(Ys, dtype=np.float32)
    L = float(np.mean(e.astype(np.float64) ** 2))
    d = bf16(np.float32(2.0 / (B * N_OUT)) * e)
    g = {"W4": _mm(h[3].T, d), "b4": d.astype(np.float64).sum(0)}
    dh = _mm(d, w["W4"].T)
    for l in (3, 2, 1):
        hl = h[l].astype(np.float32)
        dz = bf16(dh * (np.float32(1.0) - hl * hl))
        g[f"W{l}"] = _mm(h[l - 1].T, dz)
        g[f"b{l}"] = dz.astype(np.float64).sum(0)
        if l > 1:
            dh = _mm(dz, w[f"W{l}"].T)
    return L, pack(g, dtype=np.float32)
