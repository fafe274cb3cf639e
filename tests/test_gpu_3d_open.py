"""GPU parity of the three-dimensional open ends in x (non-equilibrium extrapolation at
the inlet plane x = 0 and the outlet plane x = nx - 1) against the FP64 3-D oracle,
through the C ABI (dilbm3d_*), on D3Q19 and D3Q27.

Tolerances, fixed before measuring (the bars of the periodic 3-D path):
* one step from the same random state: every population within 256 * 2^-24 of the
  largest deviation, sphere forces within 1e-4 of the largest, rho within 1e-6 and the
  velocity field (boundary planes included) within 1e-5 relative L2;
* 400 steps of an inflow channel or duct with a fixed sphere: velocity relative L2 <= 1e-5
  and drag within 1e-4 relative (FP32); 2e-3 and 2e-2 with FP16 storage;
* FP16 one step: populations within 2^-8 of the largest deviation (the FP16 bound of the
  periodic one-step tests).
"""
import numpy as np
import pytest

from oracle import binding3d as o3
from paper_2106_08950_amd import dilbm, dilbm3d, inputs3d
from helpers import log_case, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

U32 = 2.0**-24
STEP_TOL = 256 * U32

OPEN = dict(x_boundary=1, inlet_kind=0, inlet_profile=1, outlet_kind=0,
            inlet_velocity=(0.04, 0.005, -0.003), inlet_density=1.003, outlet_density=0.998)


def _pair(wl, q, storage=0, **ends):
    o = o3.Oracle3Solver(o3.Oracle3Params(
        nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, rho0=wl.rho0, eps=wl.eps, cutoff=wl.cutoff,
        G=tuple(wl.G), g=tuple(wl.g), wall_mask=wl.wall_mask, wall_h=wl.wall_h,
        force_mode=wl.force_mode, eps_p=wl.eps_p, eps_p1=wl.eps_p1, eps_w=wl.eps_w,
        eps_w1=wl.eps_w1, xi=wl.xi, lattice=q, x_boundary=ends["x_boundary"],
        inlet_kind=ends["inlet_kind"], inlet_profile=ends["inlet_profile"],
        outlet_kind=ends["outlet_kind"], u_in=tuple(ends["inlet_velocity"]),
        rho_in=ends["inlet_density"], rho_out=ends["outlet_density"]))
    g = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, lattice=q, storage=storage, **ends))
    if wl.nbodies:
        for s in (o, g):
            s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return o, g


# seed, (nx, ny, nz), walls, open-end kinds (inlet, profile, outlet); spheres sit in the
# middle of x, their supports off the boundary planes
ONE_STEP = [
    (1, (70, 12, 9), inputs3d.WALL_Y, (0, 1, 0)),       # 64-wide tiles, ragged
    (2, (260, 8, 6), inputs3d.WALL_Y | inputs3d.WALL_Z, (0, 2, 1)),  # whole rows, ragged
    (3, (64, 10, 7), 0, (1, 0, 0)),                      # density inlet, exact tiles
    (4, (129, 9, 8), inputs3d.WALL_Z, (1, 0, 1)),        # density inlet, zero gradient
]


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("seed,dims,walls,kinds", ONE_STEP)
def test_open_ends_one_step_matches_oracle(seed, dims, walls, kinds, q):
    nx, ny, nz = dims
    cx = 0.5 * nx
    sp = inputs3d.spheres([[cx, 0.5 * ny, 0.5 * nz], [cx + 9.0, 0.3 * ny, 0.6 * nz]],
                          [2.5, 2.0], [1.2, 1.5], vel=[[0.01, 0.0, 0.0], [0.0, 0.01, -0.01]],
                          fixed=[1, 0])
    wl = inputs3d.Workload3D(name=f"open{seed}", nx=nx, ny=ny, nz=nz, tau=0.6 + 0.05 * seed,
                             nsteps=1, G=(1e-5, -2e-6, 3e-6), wall_mask=walls, wall_h=2.0,
                             eps=1.0, cutoff=3.0, **sp)
    ends = dict(OPEN, inlet_kind=kinds[0], inlet_profile=kinds[1], outlet_kind=kinds[2])
    f0 = np.random.Generator(np.random.PCG64(seed)).uniform(-1e-3, 1e-3, size=(q, nz, ny, nx))
    log_case(f"3d open ends one step seed={seed} {dims} D3Q{q} walls={walls} kinds={kinds}")
    o, g = _pair(wl, q, **ends)
    o.set_populations(f0)
    g.set_populations(f0)
    o.step(1)
    g.step(1)
    fo, fg = o.get_populations(), g.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    assert err <= STEP_TOL, err
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 1e-4 * np.abs(Fo).max()
    ro, *uo = o.get_fields()
    rg, *ug = g.get_fields()
    assert np.abs(rg - ro).max() < 1e-6
    assert rel_l2(np.stack(ug), np.stack(uo)) < 1e-5
    # the boundary planes report their boundary state
    for a in range(3):
        assert np.abs(ug[a][:, :, 0] - uo[a][:, :, 0]).max() < 1e-6
        assert np.abs(ug[a][:, :, -1] - uo[a][:, :, -1]).max() < 1e-6
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_fp16_open_ends_one_step_matches_oracle(q):
    """FP16 storage: one step from a random state on whole-row tiles, a duct-profile
    inlet and a density outlet; the populations within the FP16 one-step bound of the
    periodic FP16 tests (2^-8 of the largest deviation: storage rounding dominates)."""
    nx, ny, nz = 260, 10, 8
    sp = inputs3d.spheres([[130.0, 5.0, 4.0]], [2.5], [1.2], fixed=[1])
    wl = inputs3d.Workload3D(name="open16", nx=nx, ny=ny, nz=nz, tau=0.7, nsteps=1,
                             G=(1e-5, 0.0, 0.0), wall_mask=inputs3d.WALL_Y | inputs3d.WALL_Z,
                             wall_h=2.0, eps=1.0, cutoff=3.0, **sp)
    ends = dict(OPEN, inlet_profile=2)
    f0 = np.random.Generator(np.random.PCG64(7)).uniform(-1e-3, 1e-3, size=(q, nz, ny, nx))
    log_case(f"3d FP16 open ends one step D3Q{q}")
    o, g = _pair(wl, q, storage=dilbm.STORE_FP16, **ends)
    o.set_populations(f0)
    g.set_populations(f0)
    o.step(1)
    g.step(1)
    fo, fg = o.get_populations(), g.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    assert err <= 2.0**-8, err
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    assert rel_l2(np.stack(ug), np.stack(uo)) < 2e-3
    g.close()


def _inflow(profile, walls):
    nx, ny, nz = 96, 40, 32
    sp = inputs3d.spheres([[40.0, 20.3, 16.1]], [6.0], [1.0], fixed=[1])
    return inputs3d.Workload3D(name="inflow", nx=nx, ny=ny, nz=nz, tau=0.8, nsteps=400,
                               wall_mask=walls, wall_h=3.0, **sp), \
        dict(OPEN, inlet_profile=profile, inlet_velocity=(0.03, 0.0, 0.0))


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("profile,walls", [(1, inputs3d.WALL_Y),
                                           (2, inputs3d.WALL_Y | inputs3d.WALL_Z)])
def test_inflow_past_a_fixed_sphere_matches_oracle(profile, walls, q):
    wl, ends = _inflow(profile, walls)
    log_case(f"3d inflow D3Q{q} profile={profile} walls={walls}, 400 steps")
    o, g = _pair(wl, q, **ends)
    o.step(400)
    g.step(400)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    print(f"3d inflow D3Q{q} profile {profile}: u rel L2 {e:.3e}, "
          f"drag {Fg[0, 0]:.6e} vs {Fo[0, 0]:.6e}")
    assert np.abs(uo[0]).max() > 0.02  # the inflow has arrived
    assert e < 1e-5
    assert abs(Fg[0, 0] - Fo[0, 0]) <= 1e-4 * abs(Fo[0, 0])
    g.close()


def test_density_driven_channel_matches_oracle():
    """Density inlet and zero-gradient outlet: the flow is driven by the density the inlet
    plane holds, D3Q19, 400 steps."""
    wl, _ = _inflow(1, inputs3d.WALL_Y)
    ends = dict(OPEN, inlet_kind=dilbm.INLET_PRESSURE, outlet_kind=dilbm.OUTLET_ZERO_GRADIENT,
                inlet_density=1.01)
    log_case("3d density-driven channel D3Q19, 400 steps")
    o, g = _pair(wl, 19, **ends)
    o.step(400)
    g.step(400)
    ro, *uo = o.get_fields()
    rg, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    print(f"3d density-driven channel: u rel L2 {e:.3e}")
    assert np.abs(uo[0]).max() > 1e-3
    assert e < 1e-5 and np.abs(rg - ro).max() < 1e-6
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_fp16_inflow_duct_matches_oracle(q):
    wl, ends = _inflow(2, inputs3d.WALL_Y | inputs3d.WALL_Z)
    log_case(f"3d FP16 inflow duct D3Q{q}, 400 steps")
    o, g = _pair(wl, q, storage=dilbm.STORE_FP16, **ends)
    o.step(400)
    g.step(400)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    ef = abs(Fg[0, 0] - Fo[0, 0]) / abs(Fo[0, 0])
    print(f"3d FP16 inflow duct D3Q{q}: u rel L2 {e:.3e}, drag rel error {ef:.3e}")
    assert e < 2e-3 and ef < 2e-2
    g.close()


def test_periodic_and_open_instances_agree_away_from_the_ends():
    """A solve with open ends whose boundary state is the periodic flow's own (zero
    gradient at both ends of a uniform stream) stays the uniform stream: every node keeps
    the velocity it started with."""
    nx, ny, nz, q = 80, 12, 10, 19
    wl = inputs3d.Workload3D(name="uniform", nx=nx, ny=ny, nz=nz, tau=0.7, nsteps=50)
    ends = dict(OPEN, inlet_kind=dilbm.INLET_VELOCITY, inlet_profile=0,
                outlet_kind=dilbm.OUTLET_ZERO_GRADIENT, inlet_velocity=(0.02, 0.0, 0.0))
    cx, cy, cz, w, _ = o3.lattice(q)
    feq = o3.feq(1.0, [0.02, 0.0, 0.0], q) - w
    f0 = np.broadcast_to(feq[:, None, None, None], (q, nz, ny, nx)).copy()
    log_case("3d uniform stream through open ends, 50 steps")
    g = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, lattice=q, **ends))
    g.set_populations(f0)
    g.step(50)
    _, ux, uy, uz = g.get_fields()
    assert np.abs(ux - 0.02).max() < 1e-6 and np.abs(uy).max() < 1e-6 and np.abs(uz).max() < 1e-6
    g.close()


def test_full_size_inflow_duct_one_step():
    """The 256^3 inflow duct of the benchmark (walls across y and z, duct-profile inlet,
    density outlet, 200 fixed spheres) in the launch configuration the benchmark times:
    one step from a random state, every population checked against the oracle."""
    wl = inputs3d.inflow_duct3d()
    log_case(f"3d full size {wl.name}, 1 step")
    f0 = inputs3d.random_deviations3d(wl.nx, wl.ny, wl.nz, amp=1e-4, seed=12).astype(np.float32)
    f0 = f0.astype(np.float64)  # exactly representable on the GPU
    ends = dict(x_boundary=wl.x_boundary, inlet_kind=wl.inlet_kind,
                inlet_profile=wl.inlet_profile, outlet_kind=wl.outlet_kind,
                inlet_velocity=tuple(wl.u_in), inlet_density=wl.rho_in,
                outlet_density=wl.rho_out)
    o, g = _pair(wl, 19, **ends)
    g.set_populations(f0)
    g.step(1)
    fg = g.get_populations()
    Fg, _ = g.get_particle_forces()
    g.close()
    o.set_populations(f0)
    del f0
    o.step(1)
    fo = o.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    del fg, fo
    assert err <= STEP_TOL, err
    Fo, _ = o.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 1e-4 * np.abs(Fo).max()
