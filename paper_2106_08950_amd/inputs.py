"""Seeded synthetic inputs for the DI-LBM workloads.

This module only draws numbers: problem sizes, body placements, parameters and random
population deviations.  It holds none of the method's arithmetic, so that the GPU path
and the FP64 oracle can both be fed from it without sharing any computation.

Workloads (lattice units; node (i, j) sits at (i + 0.5, j + 0.5)):

* ``cylinder_channel``   -- 200x80 channel, diffuse walls across the y seam (surfaces at
  y = 4 and y = 76), fixed disc R = 10 at (100, 40), tau = 0.8, eps = 2, body force
  G = (1e-6, 0), 2000 steps.  Stands in for the fixed-cylinder test of Section 3.1.
* ``settling_disc``      -- 400x1600 box with diffuse walls on both seams, one free disc
  R = 12.5, density ratio 1.5, g = (0, 1e-5) in the sign convention of Eq. (22), released at
  rest at (200, 1400), tau = 0.7, 20000 steps.  Stands in for the settling test of
  Section 3.2.
* ``dense_suspension``   -- 4096x4096 periodic, 2000 discs R = 8 placed by rejection
  sampling (seed 3), density ratio 1.2, G = (1e-6, 0), tau = 0.6, 5000 steps.
* ``inflow_array``       -- 4096x2048 channel open in x: uniform velocity inlet u = 0.05
  at x = 0, zero-gradient outlet, periodic across, 300 fixed discs R = 8 (seed 6) kept 64
  nodes clear of both ends, tau = 0.6.  The Section 3.1 set-up at benchmark size.
* ``ensemble``           -- 256 independent periodic solves (seed 4): nx log-uniform in
  [128, 1024], ny log-uniform in [128, 512], 1-32 discs with R uniform in [4, 16], tau
  uniform in [0.55, 1.5], G_x uniform in [1e-7, 1e-5], 2000 steps each.
* ``request_stream``     -- Poisson arrivals at 50/s (seed 5) of periodic square solves,
  side log-uniform in [64, 2048], 0-64 discs (capped by placement) with R in [4, 16],
  steps uniform in [1000, 20000], tau in [0.55, 1.5], G_x in [1e-7, 1e-5] clipped to
  0.02 / steps.

Disc placement: centres uniform over the domain; a candidate is accepted if its
minimum-image centre distance to every accepted disc is at least R_a + R_b + xi and its
distance to every wall surface is at least R + xi; after 1000 rejected candidates for one
disc the placement stops and the actual count is kept.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

WALL_Y = 1
WALL_X = 2


@dataclass
class Workload:
    """One solve: parameters, initial bodies and the number of steps."""

    name: str
    nx: int
    ny: int
    tau: float
    nsteps: int
    rho0: float = 1.0
    eps: float = 2.0
    cutoff: float = 4.0
    G: tuple = (0.0, 0.0)
    g: tuple = (0.0, 0.0)
    wall_mask: int = 0
    wall_h: float = 4.0
    force_mode: int = 0
    eps_p: float = 1.0e4
    eps_p1: float = 1.0e4
    eps_w: float = 0.5e4
    eps_w1: float = 0.5e4
    xi: float = 1.0
    x_boundary: int = 0        # 1: inlet column x = 0, outlet column x = nx - 1
    inlet_kind: int = 0        # 0 velocity, 1 pressure
    inlet_profile: int = 0     # 0 uniform, 1 parabolic across the channel
    outlet_kind: int = 0       # 0 pressure, 1 zero gradient
    u_in: tuple = (0.0, 0.0)
    rho_in: float = 1.0
    rho_out: float = 1.0
    pos: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    vel: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    omega: np.ndarray = field(default_factory=lambda: np.zeros(0))
    radius: np.ndarray = field(default_factory=lambda: np.zeros(0))
    density: np.ndarray = field(default_factory=lambda: np.zeros(0))
    fixed: np.ndarray = field(default_factory=lambda: np.zeros(0, np.uint8))

    @property
    def nbodies(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nodes(self) -> int:
        return int(self.nx) * int(self.ny)

    def with_steps(self, nsteps: int) -> "Workload":
        return replace(self, nsteps=int(nsteps))


def _bodies(pos, radius, density, vel=None, omega=None, fixed=None):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 2)
    n = pos.shape[0]
    return dict(
        pos=pos,
        vel=np.zeros((n, 2)) if vel is None else np.asarray(vel, np.float64).reshape(n, 2),
        omega=np.zeros(n) if omega is None else np.asarray(omega, np.float64).reshape(n),
        radius=np.asarray(radius, np.float64).reshape(n),
        density=np.asarray(density, np.float64).reshape(n),
        fixed=(np.zeros(n, np.uint8) if fixed is None
               else np.asarray(fixed, np.uint8).reshape(n)),
    )


def place_discs(rng, nx, ny, count, radius_fn, xi=1.0, wall_mask=0, wall_h=4.0,
                max_tries=1000):
    """Rejection-sample non-overlapping disc centres (see module docstring).

    ``radius_fn(rng)`` draws one radius.  Returns (pos [n, 2], radius [n])."""
    pos = []
    rad = []
    for _ in range(count):
        r = float(radius_fn(rng))
        placed = False
        for _try in range(max_tries):
            x = rng.uniform(0.0, nx)
            y = rng.uniform(0.0, ny)
            if wall_mask & WALL_Y and (y - wall_h < r + xi or (ny - wall_h) - y < r + xi):
                continue
            if wall_mask & WALL_X and (x - wall_h < r + xi or (nx - wall_h) - x < r + xi):
                continue
            ok = True
            if pos:
                p = np.asarray(pos)
                q = np.asarray(rad)
                dx = np.abs(p[:, 0] - x)
                dx = np.minimum(dx, nx - dx)
                dy = np.abs(p[:, 1] - y)
                dy = np.minimum(dy, ny - dy)
                ok = bool(np.all(np.hypot(dx, dy) >= q + r + xi))
            if ok:
                pos.append((x, y))
                rad.append(r)
                placed = True
                break
        if not placed:
            break
    return np.asarray(pos, np.float64).reshape(-1, 2), np.asarray(rad, np.float64)


def cylinder_channel() -> Workload:
    return Workload(name="cylinder_channel_200x80", nx=200, ny=80, tau=0.8, nsteps=2000,
                    eps=2.0, G=(1.0e-6, 0.0), wall_mask=WALL_Y, wall_h=4.0,
                    **_bodies([[100.0, 40.0]], [10.0], [1.0], fixed=[1]))


def settling_disc() -> Workload:
    return Workload(name="settling_disc_400x1600", nx=400, ny=1600, tau=0.7, nsteps=20000,
                    eps=2.0, g=(0.0, 1.0e-5), wall_mask=WALL_X | WALL_Y, wall_h=4.0,
                    **_bodies([[200.0, 1400.0]], [12.5], [1.5]))


def dense_suspension(n=4096, count=2000, seed=3) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, rad = place_discs(rng, n, n, count, lambda r: 8.0)
    return Workload(name=f"dense_suspension_{n}x{n}_{len(rad)}discs", nx=n, ny=n, tau=0.6,
                    nsteps=5000, eps=2.0, G=(1.0e-6, 0.0),
                    **_bodies(pos, rad, np.full(len(rad), 1.2)))


def inflow_array(nx=4096, ny=2048, count=300, seed=6) -> Workload:
    """A uniform stream (u = 0.05) entering at the inlet column through an array of fixed
    discs (R = 8, kept 64 nodes clear of both ends) and leaving through a zero-gradient
    outlet, periodic across: the Section 3.1 set-up at benchmark size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, rad = place_discs(rng, nx - 128, ny, count, lambda r: 8.0)
    pos = pos + np.array([64.0, 0.0])
    return Workload(name=f"inflow_array_{nx}x{ny}_{len(rad)}discs", nx=nx, ny=ny, tau=0.6,
                    nsteps=2000, eps=2.0, x_boundary=1, inlet_kind=0, outlet_kind=1,
                    u_in=(0.05, 0.0),
                    **_bodies(pos, rad, np.full(len(rad), 1.0),
                              fixed=np.ones(len(rad), np.uint8)))


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def ensemble(count=256, seed=4, nsteps=2000) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        nx = _log_uniform_int(rng, 128, 1024)
        ny = _log_uniform_int(rng, 128, 512)
        nd = int(rng.integers(1, 33))
        tau = float(rng.uniform(0.55, 1.5))
        gx = float(rng.uniform(1.0e-7, 1.0e-5))
        pos, rad = place_discs(rng, nx, ny, nd, lambda r: r.uniform(4.0, 16.0))
        out.append(Workload(name=f"ensemble_{k}", nx=nx, ny=ny, tau=tau, nsteps=nsteps,
                            eps=2.0, G=(gx, 0.0),
                            **_bodies(pos, rad, np.full(len(rad), 1.2))))
    return out


def request_stream(count=500, rate=50.0, seed=5) -> list:
    """Returns a list of (arrival_time_s, Workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        side = _log_uniform_int(rng, 64, 2048)
        nd = int(rng.integers(0, 65))
        steps = int(rng.integers(1000, 20001))
        tau = float(rng.uniform(0.55, 1.5))
        gx = min(float(rng.uniform(1.0e-7, 1.0e-5)), 0.02 / steps)
        pos, rad = place_discs(rng, side, side, nd, lambda r: r.uniform(4.0, 16.0))
        out.append((t, Workload(name=f"request_{k}", nx=side, ny=side, tau=tau, nsteps=steps,
                                eps=2.0, G=(gx, 0.0),
                                **_bodies(pos, rad, np.full(len(rad), 1.2)))))
    return out


def random_deviations(nx, ny, amp=1.0e-3, seed=0) -> np.ndarray:
    """Population deviations f_i - w_i rho0, uniform in [-amp, amp], shape [9, ny, nx]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amp, amp, size=(9, ny, nx))


def random_bodies(rng, nx, ny, count, rmin=3.0, rmax=10.0, speed=0.02, spin=1.0e-3,
                  density=1.3, allow_overlap=False, fixed_frac=0.0):
    """Random bodies for parity cases: positions, velocities and spins drawn uniformly.
    With ``allow_overlap`` the centres are unconstrained (overlapping supports)."""
    if allow_overlap:
        pos = np.stack([rng.uniform(0, nx, count), rng.uniform(0, ny, count)], axis=1)
        rad = rng.uniform(rmin, rmax, count)
    else:
        pos, rad = place_discs(rng, nx, ny, count, lambda r: r.uniform(rmin, rmax))
    n = len(rad)
    vel = rng.uniform(-speed, speed, (n, 2))
    om = rng.uniform(-spin, spin, n)
    fixed = (rng.uniform(0, 1, n) < fixed_frac).astype(np.uint8)
    return _bodies(pos, rad, np.full(n, density), vel=vel, omega=om, fixed=fixed)
