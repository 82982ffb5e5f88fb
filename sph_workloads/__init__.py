"""Seeded synthetic workloads for the WCSPH hot path.

This module only generates inputs: particle positions, velocities, masses,
types and ids, plus the run parameters that describe each workload.  It holds
none of the method's arithmetic (no kernels, neighbour search, density,
equation of state, momentum or time stepping), so both the GPU path and the
CPU oracle can take their inputs from it.

Workloads (the paper's Taylor-Green section and dam-break example describe the
geometries; the sizes are the benchmark's):

  tg64        2D Taylor-Green vortex, 64x64 lattice, periodic unit box
  tg512       2D Taylor-Green vortex, 512x512 lattice jittered by +-0.1 dx
  tg256       2D Taylor-Green vortex, 256x256 lattice (adjoint workload)
  tg1024, tg2048  the same as tg512 at 1024^2 and 2048^2 (lattice sweep)
  tg32        2D Taylor-Green vortex, 32x32 lattice (adjoint oracle companion)
  dambreak3d  3D column of water (0.4 x 0.4 x 0.8) in a 1.6 x 0.67 x 0.6 tank
              with three layers of wall particles, gravity -9.81
  cube256     3D periodic cube, 256^3 lattice jittered by +-0.2 dx, Gaussian
              random velocities with standard deviation 0.1
  dambreak2d  the paper's worked example: 2D dam break with continuity density
              and the example's Euler stage (dambreak2d_fine: the same at
              dx = 0.1/32; dambreak2d_fine_pc: with predictor-corrector steps)

Array layout is SoA: x, u have shape (dim, n) float64; m (n,) float64;
ptype (n,) uint8 (0 fluid, 1 wall); pid (n,) int32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import numpy as np

CUBIC = 0
WENDLAND = 1
QUINTIC = 2
FLUID = 0
WALL = 1
# Schemes: summation density, or continuity density (the paper's worked
# example); integrators: predictor-corrector (kick-drift-kick) steps, or the
# worked example's Euler stage (continuity only).
SUMMATION = 0
CONTINUITY = 1
PREDICTOR_CORRECTOR = 0
EULER = 1
# Cell sort keys: row-major (x fastest) or Z-order (Morton).
ROW_MAJOR, Z_ORDER = 0, 1


@dataclasses.dataclass
class Params:
    dim: int
    kernel: int            # CUBIC, WENDLAND (support 2h) or QUINTIC (support 3h)
    h: float               # smoothing length (support radius 2h)
    rho0: float
    c0: float
    nu: float
    eta: float
    dt: float
    g: Tuple[float, float, float]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    periodic: Tuple[int, int, int]
    cell_div: int = 1      # cells per support radius along an axis
    cell_order: int = 0    # sort key: ROW_MAJOR or Z_ORDER (Morton) cell keys
    scheme: int = SUMMATION
    integrator: int = PREDICTOR_CORRECTOR

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class State:
    x: np.ndarray      # (dim, n) float64
    u: np.ndarray      # (dim, n) float64
    m: np.ndarray      # (n,) float64
    ptype: np.ndarray  # (n,) uint8
    pid: np.ndarray    # (n,) int32
    rho: np.ndarray = None  # (n,) float64: initial density (continuity scheme)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    def copy(self) -> "State":
        return State(self.x.copy(), self.u.copy(), self.m.copy(), self.ptype.copy(),
                     self.pid.copy(), None if self.rho is None else self.rho.copy())


@dataclasses.dataclass
class Workload:
    name: str
    params: Params
    state: State
    steps: int
    precision: str         # "fp64" or "fp32" (pair math in FP32, FP64 integration)
    description: str


def stable_dt(h: float, c0: float, umax: float, nu: float, gmag: float) -> float:
    """Fixed time step: min(0.25 h/(c0+U), 0.125 h^2/nu, 0.25 sqrt(h/|g|))."""
    dt = 0.25 * h / (c0 + umax)
    if nu > 0:
        dt = min(dt, 0.125 * h * h / nu)
    if gmag > 0:
        dt = min(dt, 0.25 * math.sqrt(h / gmag))
    return dt


def lattice(counts, dx, origin) -> np.ndarray:
    """Cell-centred lattice: origin + (i + 1/2) dx per axis, x fastest.  (dim, n)."""
    axes = [origin[k] + (np.arange(counts[k], dtype=np.float64) + 0.5) * dx
            for k in range(len(counts))]
    grids = np.meshgrid(*axes, indexing="ij")
    # x fastest in the flattened order
    return np.stack([g.transpose().reshape(-1) for g in grids])


def taylor_green(n_side: int, jitter: float = 0.0, seed: int = 0, hdx: float = 1.3,
                 U: float = 1.0, Re: float = 100.0, kernel: int = CUBIC,
                 cell_div: int = 1) -> Tuple[Params, State]:
    """2D Taylor-Green vortex in the periodic unit box at t = 0.

    u = -U cos(2 pi x) sin(2 pi y), v = U sin(2 pi x) cos(2 pi y) evaluated at
    the (jittered) particle positions; nu = U L / Re; rho0 = 1; c0 = 10 U;
    m = rho0 dx^2.
    """
    L = 1.0
    dx = L / n_side
    x = lattice((n_side, n_side), dx, (0.0, 0.0))
    if jitter > 0:
        rng = np.random.default_rng(seed)
        x = x + rng.uniform(-jitter * dx, jitter * dx, size=x.shape)
        x = np.mod(x, L)
    u = np.empty_like(x)
    u[0] = -U * np.cos(2 * np.pi * x[0]) * np.sin(2 * np.pi * x[1])
    u[1] = U * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1])
    n = x.shape[1]
    rho0 = 1.0
    c0 = 10.0 * U
    nu = U * L / Re
    h = hdx * dx
    params = Params(dim=2, kernel=kernel, h=h, rho0=rho0, c0=c0, nu=nu, eta=0.01,
                    dt=stable_dt(h, c0, U, nu, 0.0), g=(0.0, 0.0, 0.0),
                    lo=(0.0, 0.0, 0.0), hi=(L, L, 0.0), periodic=(1, 1, 0),
                    cell_div=cell_div)
    state = State(x=x, u=u, m=np.full(n, rho0 * dx * dx), ptype=np.zeros(n, np.uint8),
                  pid=np.arange(n, dtype=np.int32))
    return params, state


def dam_break_3d(dx: float = 0.4 / 93, hdx: float = 1.3, layers: int = 3,
                 tank=(1.6, 0.67, 0.6), column=(0.4, 0.4, 0.8),
                 cell_div: int = 1) -> Tuple[Params, State]:
    """3D dam-break-like box: fluid column in the tank corner, at rest; wall
    particles fill `layers` lattice layers outside the tank floor and four
    sides (open top).  z is up, g = (0, 0, -9.81), Wendland C2, rho0 = 1000,
    c0 = 10 sqrt(2 g H) with H the column height, nu = alpha h c0 / (2(d+2))
    with alpha = 0.1.
    """
    gz = 9.81
    nfx, nfy, nfz = (int(round(c / dx)) for c in column)
    fluid = lattice((nfx, nfy, nfz), dx, (0.0, 0.0, 0.0))
    t = layers * dx
    outer_lo = (-t, -t, -t)
    cnt = (int(math.floor((tank[0] + 2 * t) / dx + 1e-9)),
           int(math.floor((tank[1] + 2 * t) / dx + 1e-9)),
           int(math.floor((tank[2] + t) / dx + 1e-9)))
    box = lattice(cnt, dx, outer_lo)
    inside = ((box[0] >= 0) & (box[0] < tank[0]) & (box[1] >= 0) & (box[1] < tank[1])
              & (box[2] >= 0))
    wall = box[:, ~inside]
    x = np.concatenate([fluid, wall], axis=1)
    nf, nw = fluid.shape[1], wall.shape[1]
    n = nf + nw
    rho0 = 1000.0
    H = column[2]
    c0 = 10.0 * math.sqrt(2 * gz * H)
    h = hdx * dx
    nu = 0.1 * h * c0 / (2 * (3 + 2))
    R = 2 * h
    lo = (-t - R, -t - R, -t - R)
    hi = (tank[0] + t + R, tank[1] + t + R, max(tank[2], column[2]) + 2 * R)
    params = Params(dim=3, kernel=WENDLAND, h=h, rho0=rho0, c0=c0, nu=nu, eta=0.01,
                    dt=stable_dt(h, c0, 0.0, nu, gz), g=(0.0, 0.0, -gz),
                    lo=lo, hi=hi, periodic=(0, 0, 0), cell_div=cell_div)
    ptype = np.concatenate([np.zeros(nf, np.uint8), np.ones(nw, np.uint8)])
    state = State(x=x, u=np.zeros_like(x), m=np.full(n, rho0 * dx ** 3), ptype=ptype,
                  pid=np.arange(n, dtype=np.int32))
    return params, state


def dam_break_2d(dx: float = 0.1, hdx: float = 1.2, rho0: float = 1000.0, c0: float = 10.0,
                 dt: float = 2e-4, block=(1.0, 2.0), layers: int = 3, tank=(4.0, 4.0),
                 kernel: int = CUBIC, cell_div: int = 1,
                 integrator: int = EULER) -> Tuple[Params, State]:
    """The paper's worked example (Section 3.2, 2D dam break).

    Every particle sits on one lattice of spacing dx through the origin
    (x = i dx, y = j dx, i and j integers).  Fluid: the lattice points of the
    block[0] x block[1] rectangle centred at (-1.5 + dx, 1 + dx), edges
    included, which at dx = 0.1 is the example's 11 x 21 = 231 particles with
    x from -1.9 to -0.9 (Section 3.2.1 prints both).  Solid: the tank whose
    interior is -L/2 < x < L/2, y > 0 (L, H = tank), walls up to y = H:
    `layers` lattice layers on and outside the floor line y = 0 and the side
    lines x = -+L/2, so the fluid starts one dx from the floor and the left
    wall.  m = rho0 dx^2, rho = rho0, u = 0, g = (0, -9.81), no viscosity,
    cubic spline h = hdx dx; continuity scheme with the given fixed dt, and
    the example's Euler stage unless another integrator is asked for."""
    cx, cy = -1.5 + dx, 1.0 + dx
    i0 = int(round((cx - 0.5 * block[0]) / dx))
    j0 = int(round((cy - 0.5 * block[1]) / dx))
    nbx, nby = int(round(block[0] / dx)) + 1, int(round(block[1] / dx)) + 1
    gi, gj = np.meshgrid(np.arange(i0, i0 + nbx), np.arange(j0, j0 + nby), indexing="ij")
    fluid = np.stack([gi.T.reshape(-1) * dx, gj.T.reshape(-1) * dx])
    L, H = tank
    il = int(round(0.5 * L / dx))       # the side lines at i = -+il
    jt = int(round(H / dx))             # walls up to j = jt
    wi, wj = np.meshgrid(np.arange(-il - layers + 1, il + layers),
                         np.arange(-layers + 1, jt + 1), indexing="ij")
    wi, wj = wi.T.reshape(-1), wj.T.reshape(-1)
    inside = (wi > -il) & (wi < il) & (wj > 0)
    wall = np.stack([wi[~inside] * dx, wj[~inside] * dx])
    x = np.concatenate([fluid, wall], axis=1)
    nf, nw = fluid.shape[1], wall.shape[1]
    n = nf + nw
    h = hdx * dx
    R = (3.0 if kernel == QUINTIC else 2.0) * h
    t = layers * dx
    params = Params(dim=2, kernel=kernel, h=h, rho0=rho0, c0=c0, nu=0.0, eta=0.01, dt=dt,
                    g=(0.0, -9.81, 0.0), lo=(-0.5 * L - t - R, -t - R, 0.0),
                    hi=(0.5 * L + t + R, H + R, 0.0), periodic=(0, 0, 0), cell_div=cell_div,
                    scheme=CONTINUITY, integrator=integrator)
    ptype = np.concatenate([np.zeros(nf, np.uint8), np.ones(nw, np.uint8)])
    state = State(x=x, u=np.zeros_like(x), m=np.full(n, rho0 * dx * dx), ptype=ptype,
                  pid=np.arange(n, dtype=np.int32), rho=np.full(n, rho0))
    return params, state


def periodic_cube(n_side: int = 256, jitter: float = 0.2, sigma_u: float = 0.1,
                  hdx: float = 1.5, seed: int = 4, cell_div: int = 1) -> Tuple[Params, State]:
    """3D periodic unit cube: jittered lattice, velocities N(0, sigma_u^2) per
    component, Wendland C2, rho0 = 1, c0 = 10 max|u|, nu = alpha h c0/(2(d+2))
    with alpha = 0.1."""
    L = 1.0
    dx = L / n_side
    rng = np.random.default_rng(seed)
    x = lattice((n_side,) * 3, dx, (0.0, 0.0, 0.0))
    x = x + rng.uniform(-jitter * dx, jitter * dx, size=x.shape)
    x = np.mod(x, L)
    u = rng.normal(0.0, sigma_u, size=x.shape)
    n = x.shape[1]
    umax = float(np.sqrt((u * u).sum(axis=0)).max())
    rho0 = 1.0
    c0 = 10.0 * umax
    h = hdx * dx
    nu = 0.1 * h * c0 / (2 * (3 + 2))
    params = Params(dim=3, kernel=WENDLAND, h=h, rho0=rho0, c0=c0, nu=nu, eta=0.01,
                    dt=stable_dt(h, c0, umax, nu, 0.0), g=(0.0, 0.0, 0.0),
                    lo=(0.0, 0.0, 0.0), hi=(L, L, L), periodic=(1, 1, 1), cell_div=cell_div)
    state = State(x=x, u=u, m=np.full(n, rho0 * dx ** 3), ptype=np.zeros(n, np.uint8),
                  pid=np.arange(n, dtype=np.int32))
    return params, state


def workload(name: str, **kw) -> Workload:
    """The named benchmark/parity workloads.  Seeds are fixed per workload."""
    if name == "tg64":
        p, s = taylor_green(64, **kw)
        return Workload(name, p, s, 50, "fp64",
                        "2D Taylor-Green 64x64 lattice, Re=100, cubic h=1.3dx, 50 steps, FP64")
    if name == "tg512":
        p, s = taylor_green(512, jitter=0.1, seed=1, **kw)
        return Workload(name, p, s, 1000, "fp32",
                        "2D Taylor-Green 512x512 lattice jittered +-0.1dx, Re=100, cubic "
                        "h=1.3dx, 1000 steps")
    if name in ("tg1024", "tg2048"):
        # the lattice sweep beyond the headline size, where the step has
        # enough particles to fill the chip
        k = int(name[2:])
        p, s = taylor_green(k, jitter=0.1, seed=1, **kw)
        return Workload(name, p, s, 200, "fp32",
                        f"2D Taylor-Green {k}x{k} lattice jittered +-0.1dx, Re=100, cubic "
                        "h=1.3dx, 200 steps")
    if name == "tg256":
        p, s = taylor_green(256, **kw)
        return Workload(name, p, s, 200, "fp32",
                        "2D Taylor-Green 256x256, 200 steps, checkpoint every 20")
    if name == "tg32":
        p, s = taylor_green(32, **kw)
        return Workload(name, p, s, 200, "fp64", "2D Taylor-Green 32x32 (adjoint companion)")
    if name == "dambreak2d":
        p, s = dam_break_2d(**kw)
        return Workload(name, p, s, 500, "fp64",
                        "2D dam break of the paper's worked example: 1 x 2 block (11 x 21 "
                        "= 231 fluid particles) in a 4 x 4 tank with 3 wall layers, dx = 0.1, "
                        "h = 1.2 dx, continuity density, Euler stage, dt = 2e-4")
    if name == "dambreak2d_fine":
        dx = 0.1 / 32
        p, s = dam_break_2d(dx=dx, dt=2e-4 / 32, **kw)
        return Workload(name, p, s, 1000, "fp32",
                        "2D dam break of the paper's worked example at dx = 0.1/32 "
                        "(321 x 641 block), dt = 2e-4/32")
    if name == "dambreak2d_fine_pc":
        dx = 0.1 / 32
        p, s = dam_break_2d(dx=dx, dt=2e-4 / 32, integrator=PREDICTOR_CORRECTOR, **kw)
        return Workload(name, p, s, 1000, "fp32",
                        "2D dam break of the paper's worked example at dx = 0.1/32 "
                        "(321 x 641 block), dt = 2e-4/32, predictor-corrector steps")
    if name == "dambreak3d":
        kw.setdefault("cell_div", 2)
        p, s = dam_break_3d(**kw)
        return Workload(name, p, s, 500, "fp32",
                        "3D dam-break box, Wendland C2 h=1.3dx, gravity, 500 steps")
    if name == "cube256":
        kw.setdefault("cell_div", 2)
        p, s = periodic_cube(**kw)
        return Workload(name, p, s, 1, "fp32",
                        "3D periodic cube 256^3 jittered +-0.2dx, Wendland C2 h=1.5dx, 1 step")
    raise KeyError(name)


def random_subset(n: int, k: int, seed: int = 123) -> np.ndarray:
    """k distinct particle indices, sorted, for sampled checks of large runs."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)
