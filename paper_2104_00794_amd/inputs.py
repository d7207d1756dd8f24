"""Seeded synthetic inputs: velocity models, Ricker wavelets, acquisition geometry.

This module holds no arithmetic of the method itself (no propagation, no
probing, no imaging).  It only draws the inputs that both the GPU library and
the FP64 oracle consume, so that the two see identical bytes.

The paper's own example (the 2D overthrust slice with ocean-bottom nodes,
Example section) ships no model or data, so the generators below stand in for
it: layered models with sinusoidal interfaces and Gaussian anomalies, and an
acquisition pattern that mirrors the paper's (sources near the surface,
receivers on a line 50 m apart).

Units: lengths in m, times in ms, velocities in km/s (= m/ms), frequencies in
kHz, squared slowness m = 1/v^2 in ms^2/m^2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np


# --------------------------------------------------------------------------- #
# wavelet
# --------------------------------------------------------------------------- #

def ricker(f_khz: float, dt: float, nt: int, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0, t0 = 1/f."""
    if t0 is None:
        t0 = 1.0 / f_khz
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f_khz * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


# --------------------------------------------------------------------------- #
# velocity models
# --------------------------------------------------------------------------- #

def two_layer_velocity(shape: Tuple[int, int], h: float, v_top: float, v_bottom: float,
                       depth: float) -> np.ndarray:
    """2D two-layer model, nodes with z >= depth get v_bottom.  shape = (nz, nx)."""
    nz, nx = shape
    z = np.arange(nz)[:, None] * h
    v = np.where(z >= depth - 1e-9, v_bottom, v_top) * np.ones((1, nx))
    return v.astype(np.float64)


def layered_velocity(shape: Sequence[int], h: float, seed: int, vmin: float, vmax: float,
                     nlayers: int = 8, nanom: int = 6) -> np.ndarray:
    """Layered model with sinusoidal interfaces and Gaussian anomalies (2D or 3D).

    shape = (nz, nx) or (nz, ny, nx).  Velocities of the layers are sorted
    draws from U(vmin, vmax) with the top layer at vmin and the bottom at vmax;
    interface i sits at depth zbar_i + A_i sin(2 pi x / L_i + phi_i) (plus a
    second sinusoid in y in 3D); anomalies scale v by 1 +- U(5, 15)% with
    Gaussian shape; the result is clipped to [vmin, vmax].
    """
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    nz = shape[0]
    Zext = (nz - 1) * h
    Xext = (shape[-1] - 1) * h
    Yext = (shape[1] - 1) * h if nd == 3 else 0.0
    zz = np.arange(nz) * h
    xx = np.arange(shape[-1]) * h
    yy = np.arange(shape[1]) * h if nd == 3 else None

    vel = np.sort(rng.uniform(vmin, vmax, nlayers))
    vel[0], vel[-1] = vmin, vmax
    zbar = np.sort(rng.uniform(0.08, 0.92, nlayers - 1)) * Zext
    if nd == 2:
        v = np.full((nz, shape[1]), vel[0])
        Z = zz[:, None]
    else:
        v = np.full(shape, vel[0])
        Z = zz[:, None, None]
    for i in range(nlayers - 1):
        A = rng.uniform(0.02, 0.06) * Zext
        L = rng.uniform(0.3, 1.0) * Xext
        phi = rng.uniform(0, 2 * math.pi)
        if nd == 2:
            surf = zbar[i] + A * np.sin(2 * math.pi * xx / L + phi)
            v = np.where(Z >= surf[None, :], vel[i + 1], v)
        else:
            Ay = rng.uniform(0.02, 0.06) * Zext
            Ly = rng.uniform(0.3, 1.0) * Yext
            phy = rng.uniform(0, 2 * math.pi)
            surf = (zbar[i] + A * np.sin(2 * math.pi * xx[None, :] / L + phi)
                    + Ay * np.sin(2 * math.pi * yy[:, None] / Ly + phy))
            v = np.where(Z >= surf[None, :, :], vel[i + 1], v)
    for _ in range(nanom):
        amp = rng.uniform(0.05, 0.15) * rng.choice([-1.0, 1.0])
        sig = rng.uniform(0.03, 0.08) * Xext
        cz = rng.uniform(0.2, 0.9) * Zext
        cx = rng.uniform(0.1, 0.9) * Xext
        if nd == 2:
            r2 = (zz[:, None] - cz) ** 2 + (xx[None, :] - cx) ** 2
        else:
            cy = rng.uniform(0.1, 0.9) * Yext
            r2 = ((zz[:, None, None] - cz) ** 2 + (yy[None, :, None] - cy) ** 2
                  + (xx[None, None, :] - cx) ** 2)
        v = v * (1.0 + amp * np.exp(-r2 / (2 * sig * sig)))
    return np.clip(v, vmin, vmax).astype(np.float64)


def smooth(m: np.ndarray, sigma_cells: float) -> np.ndarray:
    """Gaussian smoothing with edge replication (the starting model m0)."""
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(np.asarray(m, dtype=np.float64), sigma_cells, mode="nearest")


def slowness2(v: np.ndarray) -> np.ndarray:
    return 1.0 / (np.asarray(v, dtype=np.float64) ** 2)


# --------------------------------------------------------------------------- #
# workloads
# --------------------------------------------------------------------------- #

@dataclass
class Workload:
    """One complete, seeded problem: grid, models, geometry and probes."""
    name: str
    shape: Tuple[int, ...]          # physical nodes (nz, nx) or (nz, ny, nx)
    h: float
    order: int
    dt: float
    nt: int
    f_khz: float
    vmin: float
    vmax: float
    nbl: int = 20
    damp_R: float = 1e-3
    r: int = 8
    probe: str = "rademacher"
    probe_seed: int = 1
    model_seed: int = 0
    smooth_sigma: float = 5.0
    two_layer: Optional[Tuple[float, float, float]] = None   # (v_top, v_bottom, depth)
    src: List[Tuple[float, float, float]] = field(default_factory=list)
    rec: List[Tuple[float, float, float]] = field(default_factory=list)

    @property
    def nshots(self) -> int:
        return len(self.src)

    @property
    def ndim(self) -> int:
        return len(self.shape)

    @property
    def n_phys(self) -> int:
        return int(np.prod(self.shape))

    @property
    def n_pad(self) -> int:
        return int(np.prod([s + 2 * self.nbl for s in self.shape]))

    def velocity_true(self) -> np.ndarray:
        if self.two_layer is not None:
            vt, vb, depth = self.two_layer
            return two_layer_velocity(self.shape, self.h, vt, vb, depth)
        return layered_velocity(self.shape, self.h, self.model_seed, self.vmin, self.vmax)

    def models(self):
        """(m_true, m0) as float64 squared slowness."""
        mt = slowness2(self.velocity_true())
        return mt, smooth(mt, self.smooth_sigma)

    def src_pos(self) -> np.ndarray:
        return np.array(self.src, dtype=np.float64).reshape(-1, 3)

    def rec_pos(self) -> np.ndarray:
        """Same receiver spread for every shot: [S][nrec][3]."""
        r = np.array(self.rec, dtype=np.float64).reshape(-1, 3)
        return np.broadcast_to(r, (self.nshots,) + r.shape).copy()

    def wavelet(self) -> np.ndarray:
        w = ricker(self.f_khz, self.dt, self.nt)
        return np.broadcast_to(w, (self.nshots, self.nt)).copy()

    def with_(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def _line(x0, x1, dx, y, z):
    n = int(round((x1 - x0) / dx)) + 1
    return [(x0 + i * dx, y, z) for i in range(n)]


def _grid_spread(x0, x1, dx, z):
    n = int(round((x1 - x0) / dx)) + 1
    return [(x0 + i * dx, x0 + j * dx, z) for j in range(n) for i in range(n)]


def workload(name: str) -> Workload:
    """The named workloads (sizes from the measured configurations)."""
    if name == "c0_two_layer_2d":
        # 101 x 101 at 10 m, 1.5 over 2.5 km/s at 500 m, 10 Hz, 1 s, order 4.
        return Workload(name, (101, 101), 10.0, 4, 2.0, 501, 0.010, 1.5, 2.5,
                        r=8, probe="rademacher", probe_seed=1, smooth_sigma=5.0,
                        two_layer=(1.5, 2.5, 500.0),
                        src=[(500.0, 0.0, 20.0)], rec=_line(0.0, 1000.0, 10.0, 0.0, 20.0))
    if name == "c1_layered_2d_16shots":
        # 801 x 301 at 12.5 m, 16 shots, order 8, 15 Hz, 3 s records.
        return Workload(name, (301, 801), 12.5, 8, 1.25, 2401, 0.015, 1.5, 4.5,
                        r=16, probe="rademacher", probe_seed=12, model_seed=11, smooth_sigma=10.0,
                        src=[(500.0 + 600.0 * i, 0.0, 50.0) for i in range(16)],
                        rec=_line(0.0, 10000.0, 50.0, 0.0, 500.0))
    if name == "c2_autograd_2d":
        # 401 x 201 at 10 m, 4 shots, order 8, 10 Hz, 2 s, r = 32.
        return Workload(name, (201, 401), 10.0, 8, 1.0, 2001, 0.010, 1.5, 4.5,
                        r=32, probe="rademacher", probe_seed=22, model_seed=21, smooth_sigma=10.0,
                        src=[(x, 0.0, 20.0) for x in (500.0, 1500.0, 2500.0, 3500.0)],
                        rec=_line(0.0, 4000.0, 10.0, 0.0, 20.0))
    if name == "c3_layered_3d":
        # 401 x 401 x 301 at 12.5 m, 1 shot, order 8, 12 Hz, 2.5 s, r = 32.
        return Workload(name, (301, 401, 401), 12.5, 8, 1.25, 2001, 0.012, 1.5, 4.0,
                        r=32, probe="rademacher", probe_seed=32, model_seed=31, smooth_sigma=10.0,
                        src=[(2500.0, 2500.0, 50.0)], rec=_grid_spread(0.0, 5000.0, 25.0, 50.0))
    if name == "c4_layered_3d_201":
        # the serving mix's 3D request shape on its own: 201^3 at 12.5 m, 1 shot,
        # order 8, 12 Hz, 2 s, r = 32; receivers every 50 m at 25 m depth
        return Workload(name, (201, 201, 201), 12.5, 8, 1.25, 1601, 0.012, 1.5, 4.0,
                        r=32, probe="rademacher", probe_seed=52, model_seed=51, smooth_sigma=10.0,
                        src=[(1250.0, 1250.0, 25.0)], rec=_grid_spread(0.0, 2500.0, 50.0, 25.0))
    if name == "f4_fwi_2d":
        # The inversion experiment's shape on C1's grid and model: 49 shots 200 m
        # apart at 50 m depth, ocean-bottom receivers 50 m apart at 500 m depth,
        # 8 Hz Ricker, 3 s records (Example section), r = 16.
        return Workload(name, (301, 801), 12.5, 8, 1.25, 2401, 0.008, 1.5, 4.5,
                        r=16, probe="rademacher", probe_seed=42, model_seed=11, smooth_sigma=10.0,
                        src=[(200.0 * (i + 1), 0.0, 50.0) for i in range(49)],
                        rec=_line(0.0, 10000.0, 50.0, 0.0, 500.0))
    raise KeyError(name)


WORKLOADS = ("c0_two_layer_2d", "c1_layered_2d_16shots", "c2_autograd_2d", "c3_layered_3d", "c4_layered_3d_201", "f4_fwi_2d")


def small_2d(nz=40, nx=48, h=10.0, order=8, nt=180, nbl=6, nshots=2, nrec=9, seed=5, r=8,
             f_khz=0.015, probe="rademacher") -> Workload:
    """A small 2D problem for fast tests: off-grid sources and receivers."""
    rng = np.random.default_rng(seed)
    vmax = 3.0
    limit = 0.6124 if order == 4 else 0.5546
    dt = round(0.8 * limit * h / vmax, 3)
    X, Zd = (nx - 1) * h, (nz - 1) * h
    src = [(float(rng.uniform(0.2, 0.8) * X), 0.0, float(rng.uniform(0.1, 0.3) * Zd)) for _ in range(nshots)]
    rec = [(float(x), 0.0, float(rng.uniform(0.05, 0.15) * Zd)) for x in np.linspace(0.03 * X, 0.97 * X, nrec)]
    return Workload("small_2d", (nz, nx), h, order, dt, nt, f_khz, 1.5, vmax, nbl=nbl, r=r, probe=probe,
                    probe_seed=seed + 100, model_seed=seed, smooth_sigma=3.0, src=src, rec=rec)


def small_3d(nz=20, ny=22, nx=24, h=10.0, order=8, nt=90, nbl=5, nshots=1, nrec=6, seed=7, r=8,
             f_khz=0.02) -> Workload:
    """A small 3D problem for fast tests: off-grid sources and receivers."""
    rng = np.random.default_rng(seed)
    vmax = 3.0
    limit = 0.6124 * math.sqrt(2.0 / 3.0) if order == 4 else 0.4529
    dt = round(0.8 * limit * h / vmax, 3)
    X, Y, Zd = (nx - 1) * h, (ny - 1) * h, (nz - 1) * h
    src = [(float(rng.uniform(0.3, 0.7) * X), float(rng.uniform(0.3, 0.7) * Y),
            float(rng.uniform(0.1, 0.3) * Zd)) for _ in range(nshots)]
    rec = [(float(rng.uniform(0.05, 0.95) * X), float(rng.uniform(0.05, 0.95) * Y),
            float(rng.uniform(0.05, 0.2) * Zd)) for _ in range(nrec)]
    return Workload("small_3d", (nz, ny, nx), h, order, dt, nt, f_khz, 1.5, vmax, nbl=nbl, r=r,
                    probe_seed=seed + 100, model_seed=seed, smooth_sigma=2.0, src=src, rec=rec)


# --------------------------------------------------------------------------- #
# serving mix
# --------------------------------------------------------------------------- #

SERVING_SHAPES = (
    ((201, 201), 10.0),
    ((201, 401), 10.0),
    ((301, 801), 12.5),
    ((401, 1001), 12.5),
    ((201, 201, 201), 12.5),
)


def serving_workload(idx: int, seed: int, small: bool = False) -> Workload:
    """Request `idx` of a seeded serving mix: grid shape, shot count, r and the
    model seed are drawn per request; sources at the surface, receivers on a
    surface line (2D) or grid (3D).  `small` shrinks grids and records for
    tests."""
    rng = np.random.default_rng([seed, idx])
    shape, h = SERVING_SHAPES[int(rng.integers(len(SERVING_SHAPES)))]
    is3d = len(shape) == 3
    shots = 1 if is3d else int(rng.choice([1, 2, 4, 8, 16, 32]))
    r = int(rng.choice([8, 32, 64]))
    f = float(rng.uniform(0.010, 0.015))
    T = 2000.0 if h == 10.0 else 2500.0 if is3d else 3000.0
    if small:
        shape = tuple(max(24, s // 8) for s in shape)
        shots = min(shots, 4)
        T = 300.0
        f = 0.02
    vmin, vmax = 1.5, (4.0 if is3d else 4.5)
    limit = 0.4529 if is3d else 0.5546
    dt = float(np.floor(0.85 * limit * h / vmax * 100.0) / 100.0)
    nt = int(round(T / dt)) + 1
    X = (shape[-1] - 1) * h
    if is3d:
        Y = (shape[1] - 1) * h
        src = [(0.5 * X, 0.5 * Y, 2 * h)]
        step = 4 * h
        rec = [(i * step, j * step, 2 * h) for j in range(int(Y // step) + 1) for i in range(int(X // step) + 1)]
    else:
        xs = np.linspace(0.1 * X, 0.9 * X, shots)
        src = [(float(x), 0.0, 2 * h) for x in xs]
        rec = [(i * 2 * h, 0.0, 2 * h) for i in range(int(X // (2 * h)) + 1)]
    return Workload("serve_%d" % idx, tuple(shape), h, 8, dt, nt, f, vmin, vmax, nbl=20 if not small else 8,
                    r=r, probe="rademacher", probe_seed=1000 + idx, model_seed=int(rng.integers(1 << 30)),
                    smooth_sigma=6.0, src=src, rec=rec)
