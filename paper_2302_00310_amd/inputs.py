"""Seeded synthetic initial conditions for the PonD workloads.

This module is shared by the tests, the benchmark and the FP64 oracle's
drivers.  It holds no arithmetic of the PonD method itself: it only produces
primitive fields (density, velocity, pressure) on a Cartesian grid, plus the
run parameters of each workload.  Every random draw comes from
``numpy.random.Generator(PCG64(seed))``.

Workloads (shapes follow the paper's benchmark problems):

* ``sod_1d``         -- 1D Riemann tube, stands in for the 1D shock tubes of
                        Sec. V A (strong shock tube, Le Blanc).
* ``vortex_2d``      -- isentropic vortex (textbook closed-form Euler solution)
                        advected diagonally, periodic box.
* ``quadrants_2d``   -- four-quadrant piecewise-constant state drawn from a
                        seed, stands in for the 2D Riemann configuration of
                        Sec. V A.
* ``shu_osher_2d``   -- Mach-3 normal shock running into a sinusoidal density
                        field with a random phase per row, stands in for the
                        Shu--Osher problem of Sec. V C.
* ``serving_requests`` -- Poisson stream of independent solves.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Boundary-condition codes (same numbering as the C interfaces).
BC_PERIODIC = 0
BC_ZERO_GRADIENT = 1
BC_INFLOW = 2
BC_WALL = 3


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Workload:
    """Primitive initial fields plus the run parameters of one solve.

    Arrays are row-major ``[ny, nx]`` (x fastest); 1D workloads have ny = 1.
    """
    name: str
    dim: int
    nx: int
    ny: int
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    p: np.ndarray
    gamma: float = 1.4
    tau: float = 0.55          # tau1 / dt
    prandtl: float = 1.0
    cfl: float = 0.2
    dx: float = 0.0            # 0 -> 1/nx
    bc: List[int] = field(default_factory=lambda: [BC_PERIODIC] * 4)
    inflow: List[List[float]] = field(default_factory=lambda: [[1.0, 0.0, 0.0, 1.0]] * 4)
    wall: List[List[float]] = field(default_factory=lambda: [[0.0, 0.0, 1.0]] * 4)  # u_x, u_y, T
    accel: List[float] = field(default_factory=lambda: [0.0, 0.0])  # body-force acceleration
    steps: int = 1
    seed: Optional[int] = None

    @property
    def ncell(self) -> int:
        return self.nx * self.ny

    def fields(self):
        """Contiguous float64 copies of (rho, ux, uy, p), flattened x-fastest."""
        return tuple(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                     for a in (self.rho, self.ux, self.uy, self.p))


def sod_1d(nx: int = 400, steps: int = 200, tau: float = 0.55,
           prandtl: float = 1.0, gamma: float = 1.4) -> Workload:
    """Left (1, 0, 1) | right (0.125, 0, 0.1), discontinuity at x = 0.5,
    zero-gradient (outflow) ends."""
    x = (np.arange(nx) + 0.5) / nx
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)[None, :]
    p = np.where(left, 1.0, 0.1)[None, :]
    z = np.zeros((1, nx))
    return Workload("sod_1d", 1, nx, 1, rho, z.copy(), z.copy(), p, gamma=gamma,
                    tau=tau, prandtl=prandtl,
                    bc=[BC_ZERO_GRADIENT] * 4, steps=steps)


def riemann_1d(nx: int, left, right, x0: float = 0.5, steps: int = 100,
               tau: float = 0.55, gamma: float = 1.4, length: float = 1.0) -> Workload:
    """Generic 1D Riemann tube; ``left``/``right`` are (rho, u, p)."""
    x = (np.arange(nx) + 0.5) / nx * length
    lf = x < x0
    rho = np.where(lf, left[0], right[0])[None, :]
    u = np.where(lf, left[1], right[1])[None, :]
    p = np.where(lf, left[2], right[2])[None, :]
    return Workload("riemann_1d", 1, nx, 1, rho.astype(float), u.astype(float),
                    np.zeros((1, nx)), p.astype(float), gamma=gamma, tau=tau,
                    dx=length / nx, bc=[BC_ZERO_GRADIENT] * 4, steps=steps)


def vortex_2d(n: int = 256, steps: int = 1000, mach: float = 2.0, beta: float = 5.0,
              noise: float = 1e-3, seed: int = 2, tau: float = 0.55,
              prandtl: float = 0.71, gamma: float = 1.4, ny: Optional[int] = None) -> Workload:
    """Isentropic vortex of strength ``beta`` and radius L/10 at the box
    centre, on a uniform stream of Mach ``mach`` along (1,1)/sqrt(2) (free
    stream rho = 1, T = 1), periodic box [0,1]^2.  The density is then
    multiplied by (1 + noise*U[-1,1]) at fixed pressure."""
    nx = n
    ny = n if ny is None else ny
    L = 1.0
    R = L / 10.0
    xs = (np.arange(nx) + 0.5) / nx * L
    ys = (np.arange(ny) + 0.5) / nx * L
    X, Y = np.meshgrid(xs, ys)
    xb = (X - 0.5 * L) / R
    yb = (Y - 0.5 * (ny / nx) * L) / R
    r2 = xb * xb + yb * yb
    amp = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    speed = mach * math.sqrt(gamma * 1.0)
    ux = speed / math.sqrt(2.0) - amp * yb
    uy = speed / math.sqrt(2.0) + amp * xb
    if noise:
        rng = _rng(seed)
        rho = rho * (1.0 + noise * rng.uniform(-1.0, 1.0, size=rho.shape))
    return Workload("vortex_2d", 2, nx, ny, rho, ux, uy, p, gamma=gamma, tau=tau,
                    prandtl=prandtl, dx=L / nx, bc=[BC_PERIODIC] * 4,
                    steps=steps, seed=seed)


def quadrant_states(seed: int, mach_cap: float = 3.0, gamma: float = 1.4):
    """Four (rho, ux, uy, p) states, ordered NE, NW, SW, SE, each drawn from
    rho ~ U[0.1,1.5], u_x, u_y ~ U[-1.5,1.5], p ~ U[0.03,1.5] and redrawn
    until |u| / sqrt(gamma p / rho) <= mach_cap."""
    rng = _rng(seed)
    states = []
    while len(states) < 4:
        rho = rng.uniform(0.1, 1.5)
        ux = rng.uniform(-1.5, 1.5)
        uy = rng.uniform(-1.5, 1.5)
        p = rng.uniform(0.03, 1.5)
        if math.hypot(ux, uy) / math.sqrt(gamma * p / rho) <= mach_cap:
            states.append((rho, ux, uy, p))
    return states


def quadrants_2d(n: int = 2048, steps: int = 2000, seed: int = 3, tau: float = 0.55,
                 prandtl: float = 0.71, gamma: float = 1.4, mach_cap: float = 3.0,
                 ny: Optional[int] = None) -> Workload:
    """Four-quadrant piecewise-constant state on [0,1]^2 split at the centre,
    zero-gradient boundaries on all sides."""
    nx = n
    ny = n if ny is None else ny
    st = quadrant_states(seed, mach_cap, gamma)
    xs = (np.arange(nx) + 0.5) / nx
    ys = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xs, ys)
    east = X > 0.5
    north = Y > 0.5
    quad = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
    arr = np.array(st)                          # [4, 4]
    rho, ux, uy, p = (arr[quad, k] for k in range(4))
    return Workload("quadrants_2d", 2, nx, ny, rho, ux, uy, p, gamma=gamma, tau=tau,
                    prandtl=prandtl, dx=1.0 / nx, bc=[BC_ZERO_GRADIENT] * 4,
                    steps=steps, seed=seed)


def normal_shock_state(mach: float, rho1: float, p1: float, gamma: float):
    """Post-shock (rho, u, p) behind a normal shock of Mach ``mach`` moving
    into quiescent gas (rho1, 0, p1): textbook Rankine--Hugoniot relations."""
    c1 = math.sqrt(gamma * p1 / rho1)
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    u2 = 2.0 * c1 * (m2 - 1.0) / ((gamma + 1.0) * mach)
    return rho2, u2, p2


def shu_osher_2d(nx: int = 4096, ny: int = 1024, steps: int = 5000, seed: int = 4,
                 tau: float = 0.55, prandtl: float = 0.71, gamma: float = 1.4,
                 mach: float = 3.0, lx: float = 10.0, x_shock: float = 1.0,
                 k: float = 5.0, amp: float = 0.2) -> Workload:
    """Channel [0,lx] x [0, lx*ny/nx]: a Mach-``mach`` shock at x = x_shock
    runs into quiescent gas rho = 1 + amp*sin(k x + phi_row), u = 0,
    p = 1/gamma, with phi_row ~ U[0, 2 pi) per row.  Inflow (post-shock
    state) at -x, zero gradient at +x, periodic in y."""
    rng = _rng(seed)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=ny)
    dx = lx / nx
    xs = (np.arange(nx) + 0.5) * dx
    X = np.broadcast_to(xs[None, :], (ny, nx))
    p1 = 1.0 / gamma
    r2, u2, p2 = normal_shock_state(mach, 1.0, p1, gamma)
    pre = X >= x_shock
    rho = np.where(pre, 1.0 + amp * np.sin(k * X + phase[:, None]), r2)
    ux = np.where(pre, 0.0, u2)
    uy = np.zeros_like(rho)
    p = np.where(pre, p1, p2)
    inflow = [[r2, u2, 0.0, p2], [1.0, 0.0, 0.0, p1], [1.0, 0.0, 0.0, p1], [1.0, 0.0, 0.0, p1]]
    return Workload("shu_osher_2d", 2, nx, ny, rho, ux, uy, p, gamma=gamma, tau=tau,
                    prandtl=prandtl, dx=dx,
                    bc=[BC_INFLOW, BC_ZERO_GRADIENT, BC_PERIODIC, BC_PERIODIC],
                    inflow=inflow, steps=steps, seed=seed)


def uniform_2d(nx: int, ny: int, rho: float, ux: float, uy: float, p: float,
               steps: int = 10, tau: float = 0.55, prandtl: float = 1.0,
               gamma: float = 1.4) -> Workload:
    """Uniform state in a periodic box."""
    f = lambda v: np.full((ny, nx), float(v))
    return Workload("uniform_2d", 2, nx, ny, f(rho), f(ux), f(uy), f(p), gamma=gamma,
                    tau=tau, prandtl=prandtl, dx=1.0 / nx, bc=[BC_PERIODIC] * 4,
                    steps=steps)


def thermal_couette_2d(ny: int = 32, nx: int = 4, mach: float = 0.5, eckert: float = 4.0,
                       prandtl: float = 1.0, tau: float = 10.0, t_cold: float = 1.0,
                       gamma: float = 1.4, steps: int = 1000) -> Workload:
    """Thermal Couette flow (Sec. V, viscous flows): walls at y = 0 (at rest,
    T_C) and y = L = 1 (moving with u_0 = Ma sqrt(gamma T_C) along x, T_H),
    periodic in x; ny cells across the channel, dx = 1/ny.  The wall
    temperature difference follows from the Eckert number
    Ec = u_0^2 / (C_p (T_H - T_C)).  The start is the conduction profile:
    linear u_x and T, uniform pressure p = T_C."""
    cp = gamma / (gamma - 1.0)
    u0 = mach * np.sqrt(gamma * t_cold)
    t_hot = t_cold + u0 * u0 / (cp * eckert)
    y = (np.arange(ny) + 0.5) / ny
    T = np.repeat((t_cold + (t_hot - t_cold) * y)[:, None], nx, axis=1)
    ux = np.repeat((u0 * y)[:, None], nx, axis=1)
    p = np.full((ny, nx), t_cold)
    wall = [[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.0, 0.0, t_cold], [u0, 0.0, t_hot]]
    return Workload("thermal_couette_2d", 2, nx, ny, p / T, ux, np.zeros((ny, nx)), p,
                    gamma=gamma, tau=tau, prandtl=prandtl, dx=1.0 / ny,
                    bc=[BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL], wall=wall, steps=steps)


def poiseuille_2d(ny: int = 32, nx: int = 4, u_max: float = 0.05, reynolds: float = 10.0,
                  t_wall: float = 1.0, gamma: float = 1.4, steps: int = 1000) -> Workload:
    """Force-driven channel flow (Sec. V, viscous flows): walls at rest at
    y = 0 and y = L = 1 at temperature t_wall, periodic in x, ny cells across,
    dx = 1/ny, fluid at rest with rho = 1, T = t_wall.  The acceleration
    a = 8 nu u_max / L^2 along x, with nu = u_max L / Re, gives the centre
    speed u_max of the steady Navier-Stokes profile; ``tau`` (tau1 / dt) is
    left at 1 and set by the caller from nu and dt (nu = tau1 T)."""
    one = np.ones((ny, nx))
    nu = u_max / reynolds
    a = 8.0 * nu * u_max
    return Workload("poiseuille_2d", 2, nx, ny, one.copy(), 0.0 * one, 0.0 * one, t_wall * one,
                    gamma=gamma, tau=1.0, prandtl=1.0, dx=1.0 / ny,
                    bc=[BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL],
                    wall=[[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.0, 0.0, t_wall], [0.0, 0.0, t_wall]],
                    accel=[a, 0.0], steps=steps)


@dataclass
class Request:
    """One solve of the serving stream."""
    index: int
    arrival: float           # seconds after the stream starts
    workload: Workload


SERVING_SIZES = (128, 256, 512, 1024, 2048)


def serving_requests(count: int = 512, rate: float = 50.0, seed: int = 5,
                     sizes=SERVING_SIZES, step_range=(200, 2000),
                     materialize: bool = True) -> List[Request]:
    """Poisson stream of ``count`` independent 2D solves (exponential gaps of
    mean 1/rate).  Per solve (sub-seed seed*1000 + k): Mach ~ U[0.5,4],
    Pr ~ U[0.5,1], tau ~ U[0.51,0.7], steps ~ U{lo..hi}, grid side uniform
    over ``sizes``, and a 50/50 choice between an advected vortex (periodic,
    advection Mach = the draw) and four quadrants (zero gradient, Mach cap =
    the draw)."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(count):
        sub = _rng(seed * 1000 + k)
        n = int(sub.choice(np.array(sizes)))
        mach = float(sub.uniform(0.5, 4.0))
        pr = float(sub.uniform(0.5, 1.0))
        tau = float(sub.uniform(0.51, 0.7))
        steps = int(sub.integers(step_range[0], step_range[1] + 1))
        kind = int(sub.integers(0, 2))
        wseed = int(sub.integers(0, 2 ** 31 - 1))
        if not materialize:
            wl = Workload("vortex_2d" if kind == 0 else "quadrants_2d", 2, n, n,
                          None, None, None, None, tau=tau, prandtl=pr, steps=steps,
                          seed=wseed)
        elif kind == 0:
            wl = vortex_2d(n, steps, mach=mach, seed=wseed, tau=tau, prandtl=pr)
        else:
            wl = quadrants_2d(n, steps, seed=wseed, tau=tau, prandtl=pr, mach_cap=mach)
        out.append(Request(k, float(arrivals[k]), wl))
    return out


def window(wl: Workload, x0: int, y0: int, wx: int, wy: int) -> Workload:
    """Sub-grid of ``wl`` with lower corner (x0, y0) and size wx x wy.

    Periodic axes wrap around; on a non-periodic axis the window is clipped
    to the domain and keeps the true boundary condition on the clipped side.
    Window sides that lie inside the domain get zero-gradient boundaries.
    Returns the window workload and (ox, oy), the domain coordinates of the
    window's cell (0, 0)."""
    bc = list(wl.bc)
    nbc = [BC_ZERO_GRADIENT] * 4
    def axis(lo, n, size, sides):
        if bc[sides[0]] == BC_PERIODIC:
            return (np.arange(lo, lo + size) % n), (BC_ZERO_GRADIENT, BC_ZERO_GRADIENT)
        a = max(lo, 0)
        b = min(lo + size, n)
        return np.arange(a, b), (bc[sides[0]] if a == 0 else BC_ZERO_GRADIENT,
                                 bc[sides[1]] if b == n else BC_ZERO_GRADIENT)
    ix, (nbc[0], nbc[1]) = axis(x0, wl.nx, wx, (0, 1))
    if wl.dim == 2:
        iy, (nbc[2], nbc[3]) = axis(y0, wl.ny, wy, (2, 3))
    else:
        iy = np.array([0])
        nbc[2] = nbc[3] = BC_ZERO_GRADIENT
    sub = lambda a: np.ascontiguousarray(a[np.ix_(iy, ix)])
    w = Workload(wl.name + "_window", wl.dim, len(ix), len(iy), sub(wl.rho), sub(wl.ux),
                 sub(wl.uy), sub(wl.p), gamma=wl.gamma, tau=wl.tau, prandtl=wl.prandtl,
                 cfl=wl.cfl, dx=(wl.dx if wl.dx > 0 else 1.0 / wl.nx), bc=nbc,
                 inflow=[list(r) for r in wl.inflow], wall=[list(r) for r in wl.wall],
                 accel=list(wl.accel), steps=wl.steps, seed=wl.seed)
    return w, (int(ix[0]), int(iy[0]))
