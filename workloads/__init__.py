"""Seeded synthetic workloads for the CHERT hot path.

This module only draws model parameters (Thomsen parameters, Q, tilt per
class, node -> class maps, source positions).  It holds none of the method's
arithmetic, so both the HIP library's callers and the CPU oracle's tests can
use it.  Every generator is deterministic for a given seed
(numpy PCG64 with seed = 26108 * 10 + config number by default).

The configurations stand in for the paper's workloads, which are not
available: config 1 is a homogeneous TTI block, config 2 the
layered controlled benchmark, config 3 the structurally complex 2D model.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

QP, QSV, QSH = 0, 1, 2


@dataclass
class Layer:
    vp0: float
    vs0: float
    rho: float
    eps: float
    delta: float
    gamma: float
    tilt: float      # radians
    qp: float
    qs: float
    azimuth: float = 0.0

    def thomsen_args(self):
        """(vp0, vs0, rho, eps, delta, gamma, tilt, azimuth, qp, qs)"""
        return (self.vp0, self.vs0, self.rho, self.eps, self.delta, self.gamma,
                self.tilt, self.azimuth, self.qp, self.qs)


@dataclass
class Model2D:
    name: str
    nx: int
    nz: int
    hx: float
    hz: float
    layers: List[Layer]
    class_id: np.ndarray          # int32 [nz, nx]
    sources: List[int]            # node indices ix + nx * iz
    modes: tuple
    radius: int
    n_dirs: int = 360
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.nx * self.nz


def seed_for(config: int) -> int:
    return 26108 * 10 + config


def config1() -> Model2D:
    """Homogeneous viscoelastic TTI, 101 x 101 nodes at 10 m, one class,
    qP/qSV, radius 4, source at node (50, 50)."""
    L = Layer(3000.0, 1732.0, 2300.0, 0.20, 0.10, 0.15, math.radians(30.0), 60.0, 40.0)
    nx = nz = 101
    cid = np.zeros((nz, nx), np.int32)
    return Model2D("config1_homogeneous_tti_101x101", nx, nz, 10.0, 10.0, [L], cid,
                   [50 + nx * 50], (QP, QSV), 4)


def _layer_params(rng) -> Layer:
    vp = rng.uniform(2000.0, 4500.0)
    vs = vp / rng.uniform(1.6, 2.0)
    rho = rng.uniform(2000.0, 2600.0)
    eps = rng.uniform(0.0, 0.3)
    delta = rng.uniform(-0.1, 0.2)
    gamma = rng.uniform(0.0, 0.2)
    tilt = math.radians(rng.uniform(-45.0, 45.0))
    qp = rng.uniform(30.0, 150.0)
    return Layer(vp, vs, rho, eps, delta, gamma, tilt, qp, 0.6 * qp)


def config2(seed: int = None, nx: int = 401, nz: int = 201, h: float = 5.0) -> Model2D:
    """5-layer TTI, 401 x 201 nodes at 5 m.  Interfaces at depths 200 k m
    (k = 1..4, scaled to the model depth) plus seeded sine perturbations
    (amplitude <= 20 m); per-layer parameters drawn uniformly; qP/qSV/qSH,
    5 classes, radius 5, one surface source at ix = nx // 2."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    layers = [_layer_params(rng) for _ in range(5)]
    depth = (nz - 1) * h
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    cid = np.zeros((nz, nx), np.int32)
    for k in range(1, 5):
        amp = rng.uniform(0.0, 20.0)
        lam = rng.uniform(300.0, 2000.0)
        phi = rng.uniform(0.0, 2 * math.pi)
        zi = k * depth / 5.0 + amp * np.sin(2 * math.pi * x / lam + phi)
        cid += (z[:, None] > zi[None, :]).astype(np.int32)
    return Model2D(f"config2_5layer_tti_{nx}x{nz}", nx, nz, h, h, layers, cid,
                   [nx // 2], (QP, QSV, QSH), 5)


def small_layered(nx=37, nz=23, h=10.0, n_layers=3, seed=7, radius=3, tilt_max=40.0):
    """Small layered TTI model for fast parity tests (several tiles and a
    ragged tail at the default tile size)."""
    rng = np.random.default_rng(seed)
    layers = []
    for _ in range(n_layers):
        L = _layer_params(rng)
        L.tilt = math.radians(rng.uniform(-tilt_max, tilt_max))
        layers.append(L)
    z = np.arange(nz) * h
    x = np.arange(nx) * h
    cid = np.zeros((nz, nx), np.int32)
    for k in range(1, n_layers):
        zi = k * (nz - 1) * h / n_layers + 2 * h * np.sin(2 * math.pi * x / (nx * h) * (k + 1))
        cid += (z[:, None] > zi[None, :]).astype(np.int32)
    src = [int(rng.integers(0, nx)) + nx * int(rng.integers(0, 3))]
    return Model2D(f"small_layered_{nx}x{nz}", nx, nz, h, h, layers, cid, src,
                   (QP, QSV, QSH), radius)


@dataclass
class PerNodeModel:
    """Per-node Thomsen parameters (arrays [nz, nx]) on a regular grid."""
    name: str
    nx: int
    nz: int
    hx: float
    hz: float
    params: dict                 # vp0, vs0, rho, eps, delta, gamma, tilt, qp, qs
    sources: List[int]
    modes: tuple
    radius: int
    n_dirs: int = 360

    @property
    def n_nodes(self):
        return self.nx * self.nz

    def param_rows(self):
        """[n_nodes, 10] rows (vp0, vs0, rho, eps, delta, gamma, tilt,
        azimuth, qp, qs), node order ix + nx * iz."""
        p = self.params
        cols = [p["vp0"], p["vs0"], p["rho"], p["eps"], p["delta"], p["gamma"],
                p["tilt"], np.zeros_like(p["vp0"]), p["qp"], p["qs"]]
        return np.stack([c.reshape(-1) for c in cols], axis=1).astype(np.float64)

    def layers(self):
        return [Layer(*(float(v) for v in (r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[8], r[9])))
                for r in self.param_rows()]


def _smooth_field(rng, nz, nx, h, corr, lo, hi):
    """Gaussian random field with correlation length ~corr (m), mapped to
    [lo, hi] through its empirical range."""
    kz = np.fft.fftfreq(nz, d=h)[:, None]
    kx = np.fft.rfftfreq(nx, d=h)[None, :]
    spec = np.exp(-0.5 * (2 * math.pi * corr) ** 2 * (kx ** 2 + kz ** 2) / 4.0)
    noise = rng.standard_normal((nz, nx))
    f = np.fft.irfft2(np.fft.rfft2(noise) * spec, s=(nz, nx))
    f = (f - f.min()) / max(f.max() - f.min(), 1e-30)
    return lo + (hi - lo) * f


def complex_2d(nx=1701, nz=351, h=10.0, seed=None, n_layers=30, n_faults=5,
               water_m=200.0, modes=(QSV,), radius=5, src_ix=None):
    """Structurally complex 2D TTI + Q model with per-node parameters: about
    30 folded layers cut by normal faults, Vp 1500-4700 m/s increasing with
    depth (+-10 % per layer), an isotropic water layer (Q = 1000), smooth
    eps/delta/gamma fields, tilt = local layer dip, Qp 20-200 log-linear in
    depth, Qs = 0.6 Qp."""
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    X, Z = np.meshgrid(x, z)
    depth = (nz - 1) * h
    # folded interfaces: base depths + two sines
    base = np.sort(rng.uniform(water_m + 20.0, depth, n_layers))
    horizons = []
    for b in base:
        a1, a2 = rng.uniform(0, 150, 2)
        l1, l2 = rng.uniform(2000, 8000, 2)
        p1, p2 = rng.uniform(0, 2 * math.pi, 2)
        horizons.append(b + a1 * np.sin(2 * math.pi * x / l1 + p1) + a2 * np.sin(2 * math.pi * x / l2 + p2))
    horizons = np.array(horizons)                     # [L, nx]
    # normal faults: planes x = x0 + (z - z0) / tan(dip); hanging wall shifted
    shift = np.zeros((nz, nx))
    for _ in range(n_faults):
        x0 = rng.uniform(0.1, 0.9) * x[-1]
        dip = math.radians(rng.uniform(55, 70))
        throw = rng.uniform(30, 150)
        hanging = X > x0 + Z / math.tan(dip)
        shift += np.where(hanging, throw, 0.0)
    zz = Z - shift                                     # depth in the unfaulted frame
    layer = (zz[None, :, :] > horizons[:, None, :]).sum(axis=0)
    # local dip from the nearest horizon slope
    slope = np.gradient(horizons, h, axis=1)           # [L, nx]
    li = np.clip(layer - 1, 0, n_layers - 1)
    dip = np.arctan(np.take_along_axis(slope, li, axis=0)) if n_layers else np.zeros((nz, nx))
    vfac = 1.0 + rng.uniform(-0.1, 0.1, n_layers + 1)
    vp = (1600.0 + (4700.0 - 1600.0) * np.clip(zz / depth, 0, 1)) * vfac[layer]
    vp = np.clip(vp, 1500.0, 4700.0)
    vs = vp / 1.9
    rho = 1700.0 + 0.2 * vp
    eps = _smooth_field(rng, nz, nx, h, 500.0, 0.0, 0.25)
    delta = _smooth_field(rng, nz, nx, h, 500.0, -0.05, 0.15)
    gamma = _smooth_field(rng, nz, nx, h, 500.0, 0.0, 0.15)
    qp = np.exp(np.log(20.0) + (np.log(200.0) - np.log(20.0)) * np.clip(Z / depth, 0, 1))
    qs = 0.6 * qp
    water = Z < water_m
    for a, v in ((vp, 1500.0), (vs, 0.0), (rho, 1000.0), (eps, 0.0), (delta, 0.0),
                 (gamma, 0.0), (dip, 0.0), (qp, 1000.0), (qs, 1000.0)):
        a[water] = v
    params = dict(vp0=vp, vs0=vs, rho=rho, eps=eps, delta=delta, gamma=gamma, tilt=dip,
                  qp=qp, qs=qs)
    iz_src = min(int(water_m / h), nz - 1)
    ix = nx // 2 if src_ix is None else src_ix
    return PerNodeModel(f"complex2d_{nx}x{nz}", nx, nz, h, h, params, [ix + nx * iz_src],
                        tuple(modes), radius)


SHOT_GRIDS = ((401, 201), (801, 401), (1201, 301), (1701, 351))


def config4(grids=SHOT_GRIDS, sources_per_grid=32):
    """Batched shots: grids of uneven size at 10 m from the structurally
    complex generator (200 m of water kept; layers and faults scaled to the
    extent), each with its own seed, and sources_per_grid seafloor sources
    at ix = round((j + 1/2) nx / S) on the first row below the water; qP and
    qSV, radius 5."""
    out = []
    for g, (nx, nz) in enumerate(grids):
        depth = (nz - 1) * 10.0
        m = complex_2d(nx=nx, nz=nz, h=10.0, seed=seed_for(4) * 10 + g,
                       n_layers=max(5, min(30, round(30 * depth / 3500.0))),
                       n_faults=max(1, round(5 * nx / 1701)), modes=(QP, QSV), radius=5)
        iz = 20  # first row below the water
        m.sources = [int(round((j + 0.5) * nx / sources_per_grid)) + nx * iz
                     for j in range(sources_per_grid)]
        out.append(m)
    return out


def surrogate_training_rows(n, seed=None):
    """Thomsen rows [n, 10] (vp0, vs0, rho, eps, delta, gamma, tilt,
    azimuth, qp, qs) spanning the media of the layered and the structurally
    complex models: 45 % with Vs0 = Vp0 / 1.9 and the complex model's
    anisotropy and Q ranges, 45 % with the layered model's ranges, 10 %
    isotropic fluids (no shear, Q 1000); tilt uniform in [-90, 90) deg so
    the local ray angles of a full direction set are covered densely."""
    rng = np.random.default_rng(seed_for(6) if seed is None else seed)
    rows = np.zeros((n, 10))
    u = rng.random(n)
    for i in range(n):
        tilt = math.radians(rng.uniform(-90.0, 90.0))
        if u[i] < 0.45:
            vp = rng.uniform(1500.0, 4700.0)
            qp = math.exp(rng.uniform(math.log(20.0), math.log(200.0)))
            rows[i] = (vp, vp / 1.9, 1700.0 + 0.2 * vp, rng.uniform(0.0, 0.25),
                       rng.uniform(-0.05, 0.15), rng.uniform(0.0, 0.15), tilt, 0.0, qp, 0.6 * qp)
        elif u[i] < 0.9:
            L = _layer_params(rng)
            rows[i] = (L.vp0, L.vs0, L.rho, L.eps, L.delta, L.gamma, tilt, 0.0, L.qp, L.qs)
        else:
            vp = rng.uniform(1450.0, 1600.0)
            rows[i] = (vp, 0.0, 1000.0, 0.0, 0.0, 0.0, tilt, 0.0, 1000.0, 1000.0)
    return rows


def mlp_init(shapes, seed=0):
    """Initial parameters of a multilayer perceptron as one float32 vector:
    weight matrices (2-D shapes, fan_in x fan_out) uniform in
    +-sqrt(6 / (fan_in + fan_out)) (Glorot and Bengio 2010), biases zero,
    concatenated in the order given."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in shapes:
        if len(shp) == 2:
            lim = math.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, shp).reshape(-1))
        else:
            parts.append(np.zeros(shp).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def kmeans_classes(model, K, seed=0, max_iter=100):
    """Group a per-node model into K property classes, as a user of the
    class-cache method would: k-means (k-means++ seeding, Lloyd iterations)
    on the standardised (Vp0, eps, delta, gamma, tilt, log Qp) of the solid
    nodes; each class takes the mean parameters of its members.  Fluid
    nodes (Vs0 = 0) form one extra class, last.  Returns (rows [K(+1), 10]
    in param_rows order, class_id [nz, nx] int32)."""
    rows = model.param_rows()
    solid = rows[:, 1] > 0.0
    feats = np.stack([rows[:, 0], rows[:, 3], rows[:, 4], rows[:, 5], rows[:, 6],
                      np.log(rows[:, 8])], axis=1)[solid]
    mu, sd = feats.mean(0), feats.std(0)
    z = (feats - mu) / np.where(sd > 0, sd, 1.0)
    from sklearn.cluster import KMeans
    km = KMeans(n_clusters=K, init="k-means++", n_init=1, max_iter=max_iter,
                random_state=seed, algorithm="lloyd").fit(z)
    lab = km.labels_.astype(np.int32)
    crow = np.stack([rows[solid][lab == k].mean(0) for k in range(K)])
    cid = np.full(rows.shape[0], K, np.int32)
    cid[solid] = lab
    if (~solid).any():
        crow = np.concatenate([crow, rows[~solid].mean(0, keepdims=True)])
    return crow, cid.reshape(model.nz, model.nx)


@dataclass
class Model3D:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    layers: List[Layer]
    class_id: np.ndarray          # int32 [nz, ny, nx]
    sources: List[int]            # ix + nx (iy + ny iz)
    modes: tuple
    radius: int
    n_dirs: int = 41253

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz


def config5(nx=201, ny=201, nz=101, h=10.0, seed=None, n_interfaces=5, radius=3,
            sources=((50, 50, 0), (150, 50, 0), (50, 150, 0), (150, 150, 0))):
    """3D layered TTI: planar interfaces dipping up to 15 degrees with
    uniform strike, spread over the depth; per-layer parameters as in the
    layered 2D model plus an azimuth U[0, 360) deg; qP/qSV, radius 3, four
    surface sources (ix, iy, iz)."""
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    layers = []
    for _ in range(n_interfaces + 1):
        L = _layer_params(rng)
        L.azimuth = math.radians(rng.uniform(0.0, 360.0))
        layers.append(L)
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    z = np.arange(nz) * h
    X, Y = np.meshgrid(x, y)                      # [ny, nx]
    depth = (nz - 1) * h
    cid = np.zeros((nz, ny, nx), np.int32)
    for k in range(n_interfaces):
        z0 = (k + 1) * depth / (n_interfaces + 1)
        dip = math.radians(rng.uniform(0.0, 15.0))
        strike = math.radians(rng.uniform(0.0, 360.0))
        zi = z0 + math.tan(dip) * (math.cos(strike) * (X - x.mean()) +
                                   math.sin(strike) * (Y - y.mean()))
        cid += (z[:, None, None] > zi[None, :, :]).astype(np.int32)
    src = [ix + nx * (iy + ny * iz) for ix, iy, iz in sources]
    return Model3D(f"config5_3d_layered_{nx}x{ny}x{nz}", nx, ny, nz, h, layers, cid, src,
                   (QP, QSV), radius)


@dataclass
class BlockModel3D:
    name: str
    ncx: int
    ncy: int
    ncz: int
    block_n: int
    h: float                      # lattice spacing (block edge / block_n)
    layers: List[Layer]
    class_id: np.ndarray          # int32 [NZ, NY, NX] over the lattice
    sources: List[int]            # lattice nodes ix + NX (iy + NY iz)
    receivers: List[int]
    modes: tuple
    n_dirs: int = 41253

    @property
    def lattice(self):
        n = self.block_n
        return self.ncx * n + 1, self.ncy * n + 1, self.ncz * n + 1


def blocks_3d(ncx=18, ncy=18, ncz=4, block_n=3, block=160.0, seed=None, n_layers=4,
              tilt_deg=25.0, n_rcv_side=19):
    """Compact 3D TTI on the block network: 18 x 18 x 4 blocks of 160 m
    (2880 m x 2880 m laterally, 640 m deep, 1296 blocks), block_n lattice
    intervals per block edge; n_layers layers with the layered model's
    parameter ranges, every layer tilted tilt_deg with a seeded azimuth;
    interfaces at equal depths with seeded two-way sine undulations
    (amplitude <= 40 m); one surface source at the centre and a
    n_rcv_side x n_rcv_side surface receiver grid on the block corners."""
    rng = np.random.default_rng(seed_for(6) if seed is None else seed)
    layers = []
    for _ in range(n_layers):
        L = _layer_params(rng)
        L.tilt = math.radians(tilt_deg)
        L.azimuth = math.radians(rng.uniform(0.0, 360.0))
        layers.append(L)
    h = block / block_n
    NX, NY, NZ = ncx * block_n + 1, ncy * block_n + 1, ncz * block_n + 1
    x = np.arange(NX) * h
    y = np.arange(NY) * h
    z = np.arange(NZ) * h
    X, Y = np.meshgrid(x, y)                      # [NY, NX]
    depth = (NZ - 1) * h
    cid = np.zeros((NZ, NY, NX), np.int32)
    for k in range(1, n_layers):
        amp = rng.uniform(0.0, 40.0)
        lx, ly = rng.uniform(800.0, 3000.0, 2)
        px, py = rng.uniform(0.0, 2 * math.pi, 2)
        zi = k * depth / n_layers + amp * np.sin(2 * math.pi * X / lx + px) * np.cos(
            2 * math.pi * Y / ly + py)
        cid += (z[:, None, None] > zi[None, :, :]).astype(np.int32)
    src = [(NX // 2 // block_n) * block_n + NX * ((NY // 2 // block_n) * block_n)]
    step_x = max(1, ncx // (n_rcv_side - 1)) * block_n
    step_y = max(1, ncy // (n_rcv_side - 1)) * block_n
    rcv = [ix + NX * iy for iy in range(0, NY, step_y) for ix in range(0, NX, step_x)]
    return BlockModel3D(f"blocks3d_{ncx}x{ncy}x{ncz}_n{block_n}", ncx, ncy, ncz, block_n, h,
                        layers, cid, src, rcv, (QP, QSV))
