"""Seeded synthetic inputs for the split-step solver.

This module only builds inputs: grids, bathymetry, initial surface
deformations, gauge positions and the time step chosen by the Courant rule
(|lambda| dt / dx <= 1 for still water, Numerics / Difference Scheme).  It
holds none of the solver's arithmetic, so that both the CPU oracle and the
GPU library can be fed from it.

Every array is rounded to a float32-representable value and returned as
float64, so the FP32 and FP64 paths start from identical inputs.  Seeds are
14100753 + config id (ensemble member s adds 1000*s).

Conventions (paper, Running Options / Bathymetry data): depth is positive
down, negative values are land; coordinates are metres (Cartesian) or
decimal degrees (lon, lat); arrays are row-major [ny][nx] with x fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

G = 9.81
R_EARTH = 6371000.0
SEED0 = 14100753
CARTESIAN = 0
SPHERICAL = 1


@dataclasses.dataclass
class Case:
    name: str
    coord: int
    x: np.ndarray          # [nx] metres or degrees
    y: np.ndarray          # [ny]
    depth: np.ndarray      # [ny, nx] +down, negative = land
    eta0: np.ndarray       # [ny, nx]
    u0: np.ndarray
    v0: np.ndarray
    dt: float
    steps: int
    h_min: float = 0.1
    gauges: Optional[np.ndarray] = None   # [ng, 2] int32 (ix, iy), 0-based
    enclosed: Optional[List[tuple]] = None  # list of (x, y) coordinate vectors
    extra: Optional[dict] = None
    manning_n2: float = 0.0   # bottom friction (Manning n^2); 0 = off
    friction_form: int = 0    # 0: the -alpha dt term of solver2; 1: semi-implicit option

    @property
    def nx(self) -> int:
        return int(self.depth.shape[1])

    @property
    def ny(self) -> int:
        return int(self.depth.shape[0])

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def f32(a):
    """Round to float32-representable values, return float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rng(cfg_id: int, member: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED0 + cfg_id + 1000 * member))


def _smooth_noise(rng, shape, sigma_cells):
    """Unit-variance Gaussian-filtered white noise (FFT convolution)."""
    ny, nx = shape
    w = rng.standard_normal(shape)
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (math.pi * sigma_cells) ** 2 * (kx * kx + ky * ky))
    f = np.fft.irfft2(np.fft.rfft2(w) * filt, s=shape)
    f -= f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


def _spacing_metres(coord, x, y):
    """Per-node (dx, dy) in metres for the Courant rule of the generators."""
    if coord == CARTESIAN:
        dx = np.diff(x).min() if len(x) > 1 else np.inf
        dy = np.diff(y).min() if len(y) > 1 else np.inf
        return (np.full((len(y), 1), dx), np.full((len(y), 1), dy))
    k = math.pi / 180.0
    dlon = np.diff(x).min() if len(x) > 1 else np.inf
    dlat = np.diff(y).min() if len(y) > 1 else np.inf
    dx = R_EARTH * np.cos(y * k)[:, None] * dlon * k
    dy = np.full((len(y), 1), R_EARTH * dlat * k)
    return dx, dy


def cfl_dt(coord, x, y, depth, cfl=0.8, eta=None):
    """dt = cfl * min over wet nodes of min(dx, dy) / sqrt(g*h)."""
    h = depth if eta is None else depth + eta
    dx, dy = _spacing_metres(coord, x, y)
    ds = np.minimum(np.broadcast_to(dx, depth.shape), np.broadcast_to(dy, depth.shape))
    wet = h > 0
    if not wet.any():
        raise ValueError("no wet node")
    return float(cfl * np.min(ds[wet] / np.sqrt(G * h[wet])))


def _pick_nodes(rng, mask, n):
    iy, ix = np.nonzero(mask)
    if len(ix) < n:
        raise ValueError("not enough candidate gauge nodes")
    sel = rng.choice(len(ix), size=n, replace=False)
    return np.stack([ix[sel], iy[sel]], axis=1).astype(np.int32)


def _gauss(X, Y, x0, y0, sx, sy):
    return np.exp(-0.5 * (((X - x0) / sx) ** 2 + ((Y - y0) / sy) ** 2))


# --------------------------------------------------------------------------
# Config 1: 200x200 Cartesian closed basin with a central island.
# --------------------------------------------------------------------------
def config1(nx=200, ny=200, steps=1000, seed_id=1) -> Case:
    rng = _rng(seed_id)
    dx = 1000.0
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    X, Y = np.meshgrid(x, y)
    xc, yc = x[-1] / 2, y[-1] / 2
    r = np.hypot(X - xc, Y - yc)
    depth = np.minimum(1000.0, -50.0 + 1050.0 * r / 50e3)
    half = min(x[-1], y[-1]) / 2
    lim = min(50e3, 0.5 * half)
    while True:
        ox, oy = rng.uniform(-lim, lim, size=2)
        cx, cy = xc + ox, yc + oy
        far_island = math.hypot(ox, oy) >= min(30e3, 0.6 * lim)
        far_wall = min(cx, cy, x[-1] - cx, y[-1] - cy) >= min(20e3, 0.2 * half)
        if far_island and far_wall:
            break
    sigma = 10e3 if nx >= 100 else 10.0 * dx
    eta0 = 1.0 * _gauss(X, Y, cx, cy, sigma, sigma)
    eta0 = np.where(depth > 0, eta0, 0.0)
    depth, eta0 = f32(depth), f32(eta0)
    zeros = np.zeros_like(depth)
    dt = cfl_dt(CARTESIAN, x, y, depth)
    g = _pick_nodes(rng, depth >= 100.0, 5)
    return Case("C1 cartesian island basin %dx%d" % (nx, ny), CARTESIAN, f32(x), f32(y),
                depth, eta0, zeros, zeros.copy(), dt, steps, 0.1, g)


# --------------------------------------------------------------------------
# Config 2: spherical 2400x1800 at 1 arc-min, land band, shelf, slope, dipole.
# --------------------------------------------------------------------------
def _coastal_profile(i, land_cells, shelf_cells, shelf_d=150.0, deep_d=4000.0,
                     slope_cells=100, land_top=20.0, beach_cells=10):
    """Depth as a function of the cell distance i from the land edge.

    The shelf meets the land through a linear beach of `beach_cells` cells
    (shelf_d / beach_cells metres per cell): a shelf standing directly against
    the land is a cliff of shelf_d metres, which runup over it cannot pass
    stably in this scheme, and which the depth preprocessing leaves in place
    (its ratio test looks at wet neighbours only)."""
    i = np.asarray(i, dtype=np.float64)
    land = -land_top * (land_cells - i) / land_cells
    centre = land_cells + shelf_cells + slope_cells / 2.0
    sea = shelf_d + (deep_d - shelf_d) * 0.5 * (1.0 + np.tanh((i - centre) / (slope_cells / 4.0)))
    ramp = shelf_d * (i - land_cells + 1.0) / max(beach_cells, 1)
    sea = np.where(i < land_cells + beach_cells, np.minimum(sea, ramp), sea)
    return np.where(i < land_cells, land, sea)


def _dipole(X, Y, cx, cy, along_km, across_km, sep_km, a_pos, a_neg, spherical):
    """Elliptical dipole: +a_pos lobe seaward (+x), -a_neg lobe landward."""
    if spherical:
        km_lat = 111.19492664455873
        km_lon = km_lat * math.cos(math.radians(cy))
        sx, sy = across_km / km_lon, along_km / km_lat
        off = 0.5 * sep_km / km_lon
    else:
        sx, sy = across_km * 1e3, along_km * 1e3
        off = 0.5 * sep_km * 1e3
    return (a_pos * _gauss(X, Y, cx + off, cy, sx, sy)
            - a_neg * _gauss(X, Y, cx - off, cy, sx, sy))


def config2(steps=10000, scale=1, seed_id=2) -> Case:
    """scale > 1 divides the resolution (for tests); scale=1 is full size."""
    rng = _rng(seed_id)
    d = 1.0 / 60.0 * scale
    nx, ny = int(round(40.0 / d)), int(round(30.0 / d))
    x = 140.0 + np.arange(nx) * d
    y = 10.0 + np.arange(ny) * d
    X, Y = np.meshgrid(x, y)
    land, shelf, slope = 30 // scale, 100 // scale, 100 // scale
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    depth = _coastal_profile(i, land, shelf, slope_cells=max(slope, 4))
    F = _smooth_noise(rng, (ny, nx), 20.0 / scale)
    depth = np.where(depth > 0, depth * (1.0 + 0.1 * F), depth)
    cy = rng.uniform(20.0, 30.0)
    cx = x[min(nx - 1, land + shelf + slope // 2)]
    eta0 = _dipole(X, Y, cx, cy, 75.0, 25.0, 40.0, 2.0, 1.0, True)
    eta0 = np.where(depth > 0, eta0, 0.0)
    depth, eta0 = f32(depth), f32(eta0)
    zeros = np.zeros_like(depth)
    dt = cfl_dt(SPHERICAL, x, y, depth)
    g = _pick_nodes(rng, depth >= 50.0, 50)
    return Case("C2 spherical 1-arcmin %dx%d" % (nx, ny), SPHERICAL, f32(x), f32(y),
                depth, eta0, zeros, zeros.copy(), dt, steps, 0.1, g)


# --------------------------------------------------------------------------
# Config 3: ensemble of uneven Cartesian grids.
# --------------------------------------------------------------------------
def config3_member(s, steps=3000, size_scale=1.0, seed_id=3) -> Case:
    rng = _rng(seed_id, s)
    dx = 500.0
    nx = int(rng.integers(300, 1501) * size_scale)
    ny = int(rng.integers(300, 1201) * size_scale)
    nx, ny = max(nx, 24), max(ny, 24)
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    X, Y = np.meshgrid(x, y)
    edge = int(rng.integers(0, 4))            # land on W, E, S or N
    land = max(2, int(20 * size_scale))
    shelf = max(2, int(60 * size_scale))
    if edge == 0:
        i = np.arange(nx)[None, :] * np.ones((ny, 1))
    elif edge == 1:
        i = (nx - 1 - np.arange(nx))[None, :] * np.ones((ny, 1))
    elif edge == 2:
        i = np.arange(ny)[:, None] * np.ones((1, nx))
    else:
        i = (ny - 1 - np.arange(ny))[:, None] * np.ones((1, nx))
    depth = _coastal_profile(i, land, shelf, slope_cells=max(4, int(40 * size_scale)))
    amp = rng.uniform(0.5, 3.0)
    sig = rng.uniform(5e3, 20e3) * max(size_scale, 0.05)
    # offshore centre: deep water, away from the walls
    deep = depth >= 3000.0
    cand = np.argwhere(deep)
    cy_i, cx_i = cand[rng.integers(len(cand))]
    cx, cy = x[cx_i], y[cy_i]
    if rng.random() < 0.5:
        eta0 = amp * _gauss(X, Y, cx, cy, sig, sig)
    else:
        eta0 = _dipole(X, Y, cx, cy, sig / 1e3 * 3.0, sig / 1e3, 2.0 * sig / 1e3, amp, 0.5 * amp, False)
    eta0 = np.where(depth > 0, eta0, 0.0)
    depth, eta0 = f32(depth), f32(eta0)
    zeros = np.zeros_like(depth)
    dt = cfl_dt(CARTESIAN, x, y, depth)
    return Case("C3 member %d %dx%d" % (s, nx, ny), CARTESIAN, f32(x), f32(y),
                depth, eta0, zeros, zeros.copy(), dt, steps, 0.1, None)


def config3(n=64, steps=3000, size_scale=1.0) -> List[Case]:
    return [config3_member(s, steps, size_scale) for s in range(n)]


# --------------------------------------------------------------------------
# Config 4: fully wet source-inversion problem.
# --------------------------------------------------------------------------
def config4(nx=1000, ny=800, steps=3000, nsrc=20, ngauge=30, seed_id=4):
    """Returns (case with eta0 = 0, basis [nsrc, ny, nx], c_true, c0)."""
    rng = _rng(seed_id)
    dx = 500.0
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    X, Y = np.meshgrid(x, y)
    third = nx // 3
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    ramp = np.clip((i - third) / max(1.0, nx / 6.0), 0.0, 1.0)
    depth = 50.0 + (3000.0 - 50.0) * (0.5 - 0.5 * np.cos(math.pi * ramp))
    depth = depth * (1.0 + 0.05 * _smooth_noise(rng, (ny, nx), max(2.0, nx / 50.0)))
    depth = f32(depth)
    sigma = 10e3 * nx / 1000.0
    basis = []
    for _ in range(nsrc):
        cx = rng.uniform(x[nx // 2], x[int(nx * 0.9)])
        cy = rng.uniform(y[int(ny * 0.1)], y[int(ny * 0.9)])
        basis.append(f32(_gauss(X, Y, cx, cy, sigma, sigma)))
    basis = np.stack(basis)
    c_true = rng.standard_normal(nsrc)
    shelf = np.zeros_like(depth, dtype=bool)
    shelf[ny // 10: ny - ny // 10, 2: max(3, third - 2)] = True
    gauges = _pick_nodes(rng, shelf, ngauge)
    c0 = _rng(seed_id, 1).standard_normal(nsrc)
    zeros = np.zeros_like(depth)
    dt = cfl_dt(CARTESIAN, x, y, depth)
    case = Case("C4 inversion %dx%d" % (nx, ny), CARTESIAN, f32(x), f32(y), depth,
                zeros, zeros.copy(), zeros.copy(), dt, steps, 0.1, gauges)
    return case, basis, f32(c_true), f32(c0)


# --------------------------------------------------------------------------
# Config 5: large spherical grid with plane beaches and enclosed grids.
# --------------------------------------------------------------------------
def config5(steps=20000, scale=1, seed_id=5, amp=3.0) -> Case:
    rng = _rng(seed_id)
    d = 0.5 / 60.0 * scale
    nx, ny = int(round((186.0 + 2.0 / 3.0 - 120.0) / d)), int(round(50.0 / d))
    x = 120.0 + np.arange(nx) * d
    y = 0.0 + np.arange(ny) * d
    km_lat = 111.19492664455873
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    depth = _coastal_profile(i, 60 // scale, 200 // scale, slope_cells=max(4, 200 // scale))
    # straight coast segments / islands made of plane beaches, slope 1:50
    nseg = int(rng.integers(6, 11))
    yy = y[:, None] * np.ones((1, nx))
    xx = x[None, :] * np.ones((ny, 1))
    beaches = []
    for _ in range(nseg):
        cxs = rng.uniform(x[nx // 4], x[-1] - 2.0)
        cys = rng.uniform(y[ny // 8], y[-1] - 2.0)
        theta = rng.uniform(0, math.pi)
        half_len_km = rng.uniform(20.0, 120.0)
        # signed distance (m) to a segment, positive seaward of a plateau
        klon = km_lat * np.cos(np.radians(yy))
        ex = (xx - cxs) * klon
        ey = (yy - cys) * km_lat
        along = ex * math.cos(theta) + ey * math.sin(theta)
        across = -ex * math.sin(theta) + ey * math.cos(theta)
        along_c = np.clip(along, -half_len_km, half_len_km)
        dist_km = np.hypot(along - along_c, across)
        island_half_width_km = 1.5
        s = (dist_km - island_half_width_km) * 1e3
        beach = np.minimum(s / 50.0, 1e9)
        beach = np.maximum(beach, -30.0)
        depth = np.minimum(depth, beach)
        beaches.append((cxs, cys))
    F = _smooth_noise(rng, (ny, nx), 40.0 / scale)
    depth = np.where(depth > 200.0, depth * (1.0 + 0.1 * F), depth)
    X, Y = np.meshgrid(x, y)
    cy = rng.uniform(20.0, 30.0)
    cx = x[min(nx - 1, (60 + 200 + 100) // scale)]
    eta0 = _dipole(X, Y, cx, cy, 75.0, 25.0, 40.0, amp, 0.5 * amp, True)
    eta0 = np.where(depth > 0, eta0, 0.0)
    depth, eta0 = f32(depth), f32(eta0)
    zeros = np.zeros_like(depth)
    dt = cfl_dt(SPHERICAL, x, y, depth)
    g = _pick_nodes(rng, depth >= 50.0, 50)
    # 4 enclosed grids of 400x400 at 0.1 arc-min (scaled) around beaches
    enclosed = []
    de = 0.1 / 60.0 * scale
    ne = max(8, 400 // scale)
    for k in range(4):
        cxs, cys = beaches[k % len(beaches)]
        x0 = min(max(cxs - ne * de / 2, x[1]), x[-2] - ne * de)
        y0 = min(max(cys - ne * de / 2, y[1]), y[-2] - ne * de)
        enclosed.append((f32(x0 + np.arange(ne) * de), f32(y0 + np.arange(ne) * de)))
    # runup over the land: Manning n^2 = 0.0009, the value of the paper's 2-D
    # example parameter files (without friction, thin layers on the coastal
    # plain reach hundreds of m/s and the run leaves the Courant limit)
    return Case("C5 spherical 0.5-arcmin %dx%d" % (nx, ny), SPHERICAL, f32(x), f32(y),
                depth, eta0, zeros, zeros.copy(), dt, steps, 0.1, g, enclosed,
                manning_n2=0.0009)


# --------------------------------------------------------------------------
# Small fixtures for tests.
# --------------------------------------------------------------------------
def random_small(seed, nx, ny, land=True, amp=0.5, coord=CARTESIAN, dx=100.0):
    """Random tiny grid with smooth bathymetry, optional land, random state."""
    rng = np.random.Generator(np.random.PCG64(SEED0 + 7000 + seed))
    if coord == CARTESIAN:
        x = np.cumsum(np.concatenate([[0.0], dx * rng.uniform(0.7, 1.3, nx - 1)]))
        y = np.cumsum(np.concatenate([[0.0], dx * rng.uniform(0.7, 1.3, max(ny - 1, 0))]))
    else:
        x = 150.0 + np.arange(nx) * (1.0 / 60.0)
        y = -0.2 + np.arange(ny) * (1.0 / 60.0)
    base = 30.0 + 20.0 * rng.random()
    F = _smooth_noise(rng, (ny, nx), 2.0) if nx > 2 and ny > 2 else rng.standard_normal((ny, nx))
    depth = base * (1.0 + 0.3 * F)
    if land:
        ramp = np.linspace(-1.0, 1.0, nx)[None, :] * np.ones((ny, 1))
        depth = depth * 0.5 * (1 + ramp) - 8.0 * (ramp < -0.3)
    eta = amp * _smooth_noise(rng, (ny, nx), 2.0) if nx > 2 and ny > 2 else amp * rng.standard_normal((ny, nx))
    u = 0.3 * rng.standard_normal((ny, nx))
    v = 0.3 * rng.standard_normal((ny, nx))
    depth, eta, u, v = f32(depth), f32(eta), f32(u), f32(v)
    dt = cfl_dt(coord, x, y, np.maximum(depth, 1.0), cfl=0.5)
    return Case("random small %d" % seed, coord, f32(x), f32(y), depth, eta, u, v, dt, 10, 0.1)


# --------------------------------------------------------------------------
# 1-D graded grid: solitary wave on a plane beach (the canonical runup setup
# of the paper's first example: slope 1:19.85, spacing from d offshore to
# 0.1 d near the beach, h_min 0.003 m, dt 0.03 s).
# --------------------------------------------------------------------------
def beach_1d(H_over_d=0.0185, d=1.0, cot_beta=19.85, land_extent=4.0, steps=2000, dt=0.03):
    """Returns a 1-D Case (ny = 1).  The sea is at x > 0, the still shoreline
    at x = 0, land at x < 0; the wave travels toward -x."""
    toe = cot_beta * d
    gamma = math.sqrt(3.0 * H_over_d / 4.0) / d
    half = math.acosh(math.sqrt(20.0)) / gamma
    x_center = toe + half
    x_end = x_center + 2.5 * half
    xs = [-land_extent]
    while xs[-1] < x_end:
        xx = xs[-1]
        frac = min(max(xx / toe, 0.0), 1.0)
        xs.append(xx + d * (0.1 + 0.9 * frac))
    x = np.array(xs)
    depth = np.minimum(d, x / cot_beta)
    Hw = H_over_d * d
    eta = Hw / np.cosh(gamma * (x - x_center)) ** 2
    eta = np.where(depth > 0, eta, 0.0)
    u = -math.sqrt(G / d) * eta
    x, depth, eta, u = f32(x), f32(depth)[None, :], f32(eta)[None, :], f32(u)[None, :]
    return Case("1-D beach H/d=%.4f, %d nodes" % (H_over_d, len(x)), CARTESIAN, x,
                np.array([0.0]), depth, eta, u, np.zeros_like(u), dt, steps, 0.003,
                extra={"d": d, "cot_beta": cot_beta, "H": Hw})
