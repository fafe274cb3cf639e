"""GPU parity of the three-dimensional path on the D3Q27 lattice (lattice = 27) against the
FP64 3-D oracle on the same lattice, through the C ABI (dilbm3d_*).

Tolerances, fixed before measuring, as for D3Q19: one step from the same state,
populations within 256 * 2^-24 of the largest deviation, sphere force and torque within
1e-4 of the largest, positions within 1e-9; 1000 steps, velocity relative L2 <= 1e-5 and
positions within 1e-4 lattice units.
"""
import numpy as np
import pytest

from oracle import binding3d as o3
from paper_2106_08950_amd import dilbm3d, inputs3d
from helpers import log_case, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

U32 = 2.0**-24
STEP_TOL = 256 * U32
Q = 27


def oracle27(wl):
    s = o3.Oracle3Solver(o3.Oracle3Params(
        nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, rho0=wl.rho0, eps=wl.eps, cutoff=wl.cutoff,
        G=tuple(wl.G), g=tuple(wl.g), wall_mask=wl.wall_mask, wall_h=wl.wall_h,
        force_mode=wl.force_mode, eps_p=wl.eps_p, eps_p1=wl.eps_p1, eps_w=wl.eps_w,
        eps_w1=wl.eps_w1, xi=wl.xi, lattice=Q))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def gpu27(wl, **kw):
    s = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, lattice=Q, **kw))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def deviations27(nx, ny, nz, amp, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(-amp, amp, size=(Q, nz, ny, nx))


def _case(seed, dims, nsph, walls, overlap=True, amp=1e-3, rmax=6.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    sp = inputs3d.random_spheres(rng, dims, nsph, rmin=2.5, rmax=rmax, speed=0.02, spin=2e-3,
                                 allow_overlap=overlap, fixed_frac=0.25)
    wl = inputs3d.Workload3D(name=f"q27case{seed}", nx=nx, ny=ny, nz=nz,
                             tau=0.55 + 0.1 * (seed % 5), nsteps=1, G=(1e-5, -4e-6, 2e-6),
                             g=(0.0, 0.0, -2e-5), wall_mask=walls, wall_h=3.0, **sp)
    return wl, deviations27(nx, ny, nz, amp, seed)


CASES = [
    (1, (16, 16, 16), 3, 0),
    (2, (70, 9, 5), 4, inputs3d.WALL_Y),       # ragged in x and y
    (4, (64, 8, 12), 5, 7),                    # walls on every axis
    (5, (40, 12, 1), 2, 0),                    # a single z layer
    (7, (200, 6, 5), 4, inputs3d.WALL_Y),      # whole-row tiles, one partial
    (8, (300, 5, 4), 5, 6),                    # whole-row tiles, the second ragged
]


def _check_one_step(wl, f0):
    o = oracle27(wl)
    o.set_populations(f0)
    o.step(1)
    g = gpu27(wl)
    g.set_populations(f0)
    assert np.allclose(g.get_populations(), f0, rtol=0, atol=U32 * np.abs(f0).max())
    g.step(1)
    fo = o.get_populations()
    fg = g.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    assert err <= STEP_TOL, err
    Fo, To = o.get_particle_forces()
    Fg, Tg = g.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 1e-4 * max(np.abs(Fo).max(), 1e-30)
    assert np.abs(Tg - To).max() <= 1e-4 * max(np.abs(To).max(), 1e-30)
    if wl.wall_mask:
        Wo, Wg = o.get_wall_force(), g.get_wall_force()
        assert np.abs(Wg - Wo).max() <= 1e-4 * np.abs(Wo).max()
    xo, uo, wo = o.get_particles()
    xg, ug, wg = g.get_particles()
    assert np.abs(xg - xo).max() < 1e-9
    assert np.abs(ug - uo).max() <= 1e-4 * max(np.abs(uo).max(), 1e-30) + 1e-15
    assert np.abs(wg - wo).max() <= 1e-4 * max(np.abs(wo).max(), 1e-30) + 1e-15
    ro, *uo_ = o.get_fields()
    rg, *ug_ = g.get_fields()
    assert np.abs(rg - ro).max() < 1e-6
    assert rel_l2(np.stack(ug_), np.stack(uo_)) < 1e-5
    g.close()


@pytest.mark.parametrize("seed,dims,nsph,walls", CASES)
def test_d3q27_one_step_matches_oracle(seed, dims, nsph, walls):
    wl, f0 = _case(seed, dims, nsph, walls)
    log_case(f"D3Q27 one step seed={seed} {dims} spheres={wl.nbodies} walls={walls}")
    _check_one_step(wl, f0)


@pytest.mark.parametrize("seed,dims,nsph,walls", [(11, (64, 40, 32), 6, 0),
                                                  (13, (200, 24, 16), 6, inputs3d.WALL_Z)])
def test_d3q27_many_steps_match_oracle(seed, dims, nsph, walls):
    wl, f0 = _case(seed, dims, nsph, walls, overlap=False, amp=2e-4, rmax=5.0)
    log_case(f"D3Q27 1000 steps seed={seed} {dims} spheres={wl.nbodies} walls={walls}")
    o = oracle27(wl)
    o.set_populations(f0)
    g = gpu27(wl)
    g.set_populations(f0)
    o.step(1000)
    g.step(1000)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    print(f"D3Q27 1000 steps {dims}: u rel L2 {e:.3e}")
    assert e < 1e-5
    xo, _, _ = o.get_particles()
    xg, _, _ = g.get_particles()
    d = np.abs(xg - xo)
    d = np.minimum(d, np.array(dims) - d)
    assert d.max() < 1e-4
    g.close()


def test_d3q27_channel_with_fixed_sphere():
    wl = inputs3d.channel3d()
    log_case("D3Q27 channel 96x48x32, fixed sphere, 500 steps")
    o = oracle27(wl)
    g = gpu27(wl)
    o.step(500)
    g.step(500)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    print(f"D3Q27 channel: u rel L2 {e:.3e}, drag {Fg[0, 0]:.6e} vs {Fo[0, 0]:.6e}")
    assert e < 1e-5
    assert abs(Fg[0, 0] - Fo[0, 0]) <= 1e-4 * abs(Fo[0, 0])
    g.close()


def test_d3q27_rest_state_bitwise():
    sp = inputs3d.spheres([[10.0, 10.0, 12.0], [30.0, 10.0, 12.0]], [4.0, 5.0], [1.0, 1.0])
    wr = inputs3d.Workload3D(name="rest", nx=48, ny=20, nz=24, tau=0.7, nsteps=1,
                             g=(0.0, 0.0, -1e-5), **sp)
    log_case("D3Q27 rest")
    g = gpu27(wr)
    g.step(50)
    assert not g.get_populations().any()
    x, u, w = g.get_particles()
    assert np.array_equal(x, wr.pos) and not u.any() and not w.any()
    g.close()


def test_d3q27_full_size_suspension_one_step():
    """256^3 with 400 spheres on D3Q27, in the launch configuration the benchmark times: one
    step from a random state, every population checked against the oracle."""
    wl = inputs3d.suspension3d()
    log_case(f"D3Q27 full size {wl.name}, 1 step")
    f0 = deviations27(wl.nx, wl.ny, wl.nz, 1e-4, 19).astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(20))
    wl.vel = rng.uniform(-0.01, 0.01, wl.vel.shape)
    wl.omega = rng.uniform(-1e-3, 1e-3, wl.omega.shape)
    g = gpu27(wl)
    g.set_populations(f0)
    g.step(1)
    fg = g.get_populations()
    Fg, Tg = g.get_particle_forces()
    g.close()
    o = oracle27(wl)
    o.set_populations(f0)
    del f0
    o.step(1)
    fo = o.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    del fg, fo
    assert err <= STEP_TOL, err
    Fo, To = o.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 1e-4 * np.abs(Fo).max()
    assert np.abs(Tg - To).max() <= 1e-4 * np.abs(To).max()
