"""Seeded synthetic inputs for the three-dimensional DI-LBM workloads (D3Q19, spheres).

Like ``inputs``, this module only draws numbers (sizes, sphere placements, parameters,
random population deviations) and holds none of the method's arithmetic, so the GPU path
and the FP64 oracle can both be fed from it.

Workloads (lattice units; node (i, j, k) sits at (i + 0.5, j + 0.5, k + 0.5)):

* ``suspension3d``  -- 256^3 periodic, 400 spheres R = 8 placed by rejection sampling
  (seed 8; about 5% solid volume), density ratio 1.2, G = (1e-6, 0, 0), tau = 0.6.  The
  same number of nodes as the 4096^2 two-dimensional suspension.
* ``channel3d``     -- 96 x 48 x 32 channel with diffuse walls across the y seam
  (surfaces at y = 4 and y = 44), periodic in x and z, one fixed sphere R = 8 at the
  centre, G = (1e-5, 0, 0), tau = 0.8.

Sphere placement: centres uniform over the domain; a candidate is accepted if its
minimum-image centre distance to every accepted sphere is at least R_a + R_b + xi and
its distance to every wall surface is at least R + xi; after 1000 rejected candidates
for one sphere the placement stops and the actual count is kept.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

WALL_Y = 1
WALL_X = 2
WALL_Z = 4


@dataclass
class Workload3D:
    """One 3-D solve: parameters, initial spheres and the number of steps."""

    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    nsteps: int
    rho0: float = 1.0
    eps: float = 2.0
    cutoff: float = 4.0
    G: tuple = (0.0, 0.0, 0.0)
    g: tuple = (0.0, 0.0, 0.0)
    wall_mask: int = 0
    wall_h: float = 4.0
    force_mode: int = 0
    eps_p: float = 1.0e4
    eps_p1: float = 1.0e4
    eps_w: float = 0.5e4
    eps_w1: float = 0.5e4
    xi: float = 1.0
    # open ends in x (non-equilibrium extrapolation; 0 = periodic)
    x_boundary: int = 0
    inlet_kind: int = 0
    inlet_profile: int = 0
    outlet_kind: int = 0
    u_in: tuple = (0.0, 0.0, 0.0)
    rho_in: float = 1.0
    rho_out: float = 1.0
    pos: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    vel: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    omega: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    radius: np.ndarray = field(default_factory=lambda: np.zeros(0))
    density: np.ndarray = field(default_factory=lambda: np.zeros(0))
    fixed: np.ndarray = field(default_factory=lambda: np.zeros(0, np.uint8))

    @property
    def nbodies(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nodes(self) -> int:
        return int(self.nx) * int(self.ny) * int(self.nz)

    def with_steps(self, nsteps: int) -> "Workload3D":
        return replace(self, nsteps=int(nsteps))


def spheres(pos, radius, density, vel=None, omega=None, fixed=None) -> dict:
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    return dict(
        pos=pos,
        vel=np.zeros((n, 3)) if vel is None else np.asarray(vel, np.float64).reshape(n, 3),
        omega=np.zeros((n, 3)) if omega is None else np.asarray(omega, np.float64).reshape(n, 3),
        radius=np.asarray(radius, np.float64).reshape(n),
        density=np.asarray(density, np.float64).reshape(n),
        fixed=np.zeros(n, np.uint8) if fixed is None else np.asarray(fixed, np.uint8).reshape(n),
    )


def place_spheres(rng, dims, count, radius_fn, xi=1.0, wall_mask=0, wall_h=4.0,
                  max_tries=1000):
    """Rejection-sample non-overlapping sphere centres (see module docstring)."""
    dims = np.asarray(dims, np.float64)
    wall_axes = [a for a, bit in ((1, WALL_Y), (0, WALL_X), (2, WALL_Z)) if wall_mask & bit]
    pos, rad = [], []
    for _ in range(count):
        r = float(radius_fn(rng))
        placed = False
        for _try in range(max_tries):
            c = rng.uniform(0.0, 1.0, 3) * dims
            if any(c[a] - wall_h < r + xi or (dims[a] - wall_h) - c[a] < r + xi
                   for a in wall_axes):
                continue
            if pos:
                d = np.abs(np.asarray(pos) - c)
                d = np.minimum(d, dims - d)
                if not np.all(np.sqrt((d * d).sum(axis=1)) >= np.asarray(rad) + r + xi):
                    continue
            pos.append(c)
            rad.append(r)
            placed = True
            break
        if not placed:
            break
    return np.asarray(pos, np.float64).reshape(-1, 3), np.asarray(rad, np.float64)


def suspension3d(n=256, count=400, seed=8) -> Workload3D:
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, rad = place_spheres(rng, (n, n, n), count, lambda r: 8.0)
    return Workload3D(name=f"suspension3d_{n}^3_{len(rad)}spheres", nx=n, ny=n, nz=n,
                      tau=0.6, nsteps=2000, G=(1.0e-6, 0.0, 0.0),
                      **spheres(pos, rad, np.full(len(rad), 1.2)))


def inflow_duct3d(n=256, count=200, seed=9) -> Workload3D:
    """A square duct (diffuse walls across the y and z seams) with a parabolic velocity
    inlet at x = 0 and a density outlet at x = nx - 1, past fixed spheres of radius 8
    whose supports stay 12 planes or more from the two ends."""
    rng = np.random.Generator(np.random.PCG64(seed))
    margin = 8.0 + 8.0 + 12.0
    pos, rad = place_spheres(rng, (n - 2 * margin, n, n), count, lambda r: 8.0,
                             wall_mask=WALL_Y | WALL_Z, wall_h=4.0)
    pos[:, 0] += margin
    return Workload3D(name=f"inflow_duct3d_{n}^3_{len(rad)}spheres", nx=n, ny=n, nz=n,
                      tau=0.6, nsteps=2000, wall_mask=WALL_Y | WALL_Z, wall_h=4.0,
                      x_boundary=1, inlet_kind=0, inlet_profile=2, outlet_kind=0,
                      u_in=(0.03, 0.0, 0.0), rho_in=1.0, rho_out=1.0,
                      **spheres(pos, rad, np.full(len(rad), 1.2), fixed=np.ones(len(rad))))


def ensemble3d(count=256, seed=6, nsteps=400) -> list:
    """Independent 3-D solves for the batched form: sides 32-96 (log-uniform; rows under
    192 nodes, so every member takes 64 x 4 x 1 tiles), 1-3 free spheres of radius 3.5-5,
    tau 0.6-1.2, a body force in x."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        dims = [int(round(np.exp(rng.uniform(np.log(32), np.log(96))))) for _ in range(3)]
        pos, rad = place_spheres(rng, dims, int(rng.integers(1, 4)), lambda r: r.uniform(3.5, 5.0))
        out.append(Workload3D(name=f"ensemble3d_{k}", nx=dims[0], ny=dims[1], nz=dims[2],
                              tau=float(rng.uniform(0.6, 1.2)), nsteps=nsteps,
                              G=(float(rng.uniform(1e-7, 5e-6)), 0.0, 0.0),
                              **spheres(pos, rad, np.full(len(rad), 1.2))))
    return out


def channel3d() -> Workload3D:
    return Workload3D(name="channel3d_96x48x32", nx=96, ny=48, nz=32, tau=0.8, nsteps=1000,
                      G=(1.0e-5, 0.0, 0.0), wall_mask=WALL_Y, wall_h=4.0,
                      **spheres([[48.0, 24.0, 16.0]], [8.0], [1.0], fixed=[1]))


def random_spheres(rng, dims, count, rmin=3.0, rmax=8.0, speed=0.02, spin=1.0e-3,
                   density=1.3, allow_overlap=False, fixed_frac=0.0, wall_mask=0,
                   wall_h=4.0) -> dict:
    """Random spheres for parity cases: positions, velocities and spins drawn uniformly.
    With ``allow_overlap`` the centres are unconstrained (overlapping supports)."""
    dims = np.asarray(dims, np.float64)
    if allow_overlap:
        pos = rng.uniform(0.0, 1.0, (count, 3)) * dims
        rad = rng.uniform(rmin, rmax, count)
    else:
        pos, rad = place_spheres(rng, dims, count, lambda r: r.uniform(rmin, rmax),
                                 wall_mask=wall_mask, wall_h=wall_h)
    n = len(rad)
    vel = rng.uniform(-speed, speed, (n, 3))
    om = rng.uniform(-spin, spin, (n, 3))
    fixed = (rng.uniform(0, 1, n) < fixed_frac).astype(np.uint8)
    return spheres(pos, rad, np.full(n, density), vel=vel, omega=om, fixed=fixed)


def random_deviations3d(nx, ny, nz, amp=1.0e-3, seed=0) -> np.ndarray:
    """Population deviations f_i - w_i rho0, uniform in [-amp, amp], shape [19, nz, ny, nx]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amp, amp, size=(19, nz, ny, nx))
