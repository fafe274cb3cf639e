"""GPU parity of the three-dimensional DI-LBM path (D3Q19, spheres) against the FP64 3-D
oracle, through the C ABI (dilbm3d_*).

Tolerances, fixed before measuring (the FP32 bar of the two-dimensional path):
* one step from the same state: populations within 256 * 2^-24 of the largest deviation,
  sphere force and torque within 1e-4 of the largest, positions within 1e-9;
* 1000 steps: velocity relative L2 <= 1e-5, positions within 1e-4 lattice units.
"""
import numpy as np
import pytest

from oracle import binding3d as o3
from paper_2106_08950_amd import dilbm, dilbm3d, inputs3d
from helpers import log_case, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

U32 = 2.0**-24
STEP_TOL = 256 * U32


def oracle3(wl):
    s = o3.Oracle3Solver(o3.Oracle3Params(
        nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, rho0=wl.rho0, eps=wl.eps, cutoff=wl.cutoff,
        G=tuple(wl.G), g=tuple(wl.g), wall_mask=wl.wall_mask, wall_h=wl.wall_h,
        force_mode=wl.force_mode, eps_p=wl.eps_p, eps_p1=wl.eps_p1, eps_w=wl.eps_w,
        eps_w1=wl.eps_w1, xi=wl.xi))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def gpu3(wl, **kw):
    s = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, **kw))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def vel_l2(a, b):
    return rel_l2(np.stack(a), np.stack(b))


def _case(seed, dims, nsph, walls, overlap=True, amp=1e-3, rmax=6.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    sp = inputs3d.random_spheres(rng, dims, nsph, rmin=2.5, rmax=rmax, speed=0.02, spin=2e-3,
                                 allow_overlap=overlap, fixed_frac=0.25)
    wl = inputs3d.Workload3D(name=f"case{seed}", nx=nx, ny=ny, nz=nz, tau=0.55 + 0.1 * (seed % 5),
                             nsteps=1, G=(1e-5, -4e-6, 2e-6), g=(0.0, 0.0, -2e-5),
                             wall_mask=walls, wall_h=3.0, **sp)
    return wl, inputs3d.random_deviations3d(nx, ny, nz, amp=amp, seed=seed)


CASES = [
    # seed, (nx, ny, nz), spheres, walls
    (1, (16, 16, 16), 3, 0),
    (2, (70, 9, 5), 4, inputs3d.WALL_Y),          # ragged in x and y
    (3, (130, 13, 7), 6, inputs3d.WALL_Z),        # three x tiles, ragged
    (4, (64, 8, 12), 5, 7),                       # exact tiles, walls on every axis
    (5, (40, 12, 1), 2, 0),                       # a single z layer
    (6, (33, 30, 20), 8, inputs3d.WALL_X),
    (7, (200, 6, 5), 4, inputs3d.WALL_Y),         # whole-row tiles, one partial
    (8, (300, 5, 4), 5, 6),                       # whole-row tiles, the second ragged
]


@pytest.mark.parametrize("seed,dims,nsph,walls", CASES)
def test_one_step_matches_oracle(seed, dims, nsph, walls):
    wl, f0 = _case(seed, dims, nsph, walls)
    log_case(f"3d one step seed={seed} {dims} spheres={wl.nbodies} walls={walls}")
    _check_one_step(wl, f0)


def test_one_step_spheres_on_wave_seams():
    """Whole-row tiles (nx = 260: the second tile ragged) with supports that straddle the
    seams between the 64-node waves of a row and the periodic x boundary, overlapping near
    x = 0: every wave a support reaches must take the sphere."""
    nx, ny, nz = 260, 10, 6
    sp = inputs3d.spheres(
        [[63.9, 5.0, 3.0], [0.3, 2.0, 0.5], [128.0, 8.7, 5.5], [192.05, 5.0, 3.0],
         [259.6, 7.0, 2.0], [255.7, 1.0, 4.0]],
        [3.0, 2.5, 4.0, 3.5, 3.0, 2.0], [1.2] * 6,
        vel=[[0.01, 0.0, 0.0], [0.0, -0.01, 0.0], [0.0, 0.0, 0.01], [-0.01, 0.0, 0.0],
             [0.0, 0.01, 0.0], [0.0, 0.0, -0.01]])
    wl = inputs3d.Workload3D(name="seams", nx=nx, ny=ny, nz=nz, tau=0.7, nsteps=1,
                             G=(1e-5, 0.0, 0.0), **sp)
    log_case(f"3d one step, spheres on wave seams, {(nx, ny, nz)}")
    _check_one_step(wl, inputs3d.random_deviations3d(nx, ny, nz, amp=1e-3, seed=41))


def _check_one_step(wl, f0):
    walls = wl.wall_mask
    o = oracle3(wl)
    o.set_populations(f0)
    o.step(1)
    g = gpu3(wl)
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
    if walls:
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
    assert vel_l2(ug_, uo_) < 1e-5
    g.close()


@pytest.mark.parametrize("seed,dims,nsph,walls", [(11, (64, 40, 32), 6, 0),
                                                  (12, (50, 44, 36), 5, inputs3d.WALL_Y),
                                                  (13, (200, 24, 16), 6, inputs3d.WALL_Z)])
def test_many_steps_match_oracle(seed, dims, nsph, walls):
    """The FP32 bar: 1000 steps of free spheres in a driven flow."""
    wl, f0 = _case(seed, dims, nsph, walls, overlap=False, amp=2e-4, rmax=5.0)
    log_case(f"3d 1000 steps seed={seed} {dims} spheres={wl.nbodies} walls={walls}")
    o = oracle3(wl)
    o.set_populations(f0)
    g = gpu3(wl)
    g.set_populations(f0)
    o.step(1000)
    g.step(1000)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = vel_l2(ug, uo)
    print(f"3d 1000 steps {dims}: u rel L2 {e:.3e}")
    assert e < 1e-5
    xo, _, _ = o.get_particles()
    xg, _, _ = g.get_particles()
    d = np.abs(xg - xo)
    d = np.minimum(d, np.array(dims) - d)
    assert d.max() < 1e-4


def test_channel_with_fixed_sphere():
    wl = inputs3d.channel3d()
    log_case("3d channel 96x48x32, fixed sphere, 500 steps")
    o = oracle3(wl)
    g = gpu3(wl)
    o.step(500)
    g.step(500)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = vel_l2(ug, uo)
    Fo, To = o.get_particle_forces()
    Fg, Tg = g.get_particle_forces()
    print(f"3d channel: u rel L2 {e:.3e}, drag {Fg[0, 0]:.6e} vs {Fo[0, 0]:.6e}")
    assert e < 1e-5
    assert abs(Fg[0, 0] - Fo[0, 0]) <= 1e-4 * abs(Fo[0, 0])
    Wo, Wg = o.get_wall_force(), g.get_wall_force()
    assert abs(Wg[0] - Wo[0]) <= 1e-4 * abs(Wo[0])


@pytest.mark.parametrize("dims,walls", [((48, 20, 24), 0),
                                         ((300, 6, 10), inputs3d.WALL_Y | inputs3d.WALL_Z)])
def test_fluid_only(dims, walls):
    """Without spheres; rows of 192 nodes or more run as whole-row tiles (a partial second
    tile here)."""
    nx, ny, nz = dims
    wl = inputs3d.Workload3D(name="fluid", nx=nx, ny=ny, nz=nz, tau=0.7, nsteps=1,
                             G=(2e-5, 1e-5, -5e-6), wall_mask=walls, wall_h=2.0)
    log_case(f"3d fluid only {dims} walls={walls}, 100 steps")
    o = oracle3(wl)
    g = gpu3(wl)
    f0 = inputs3d.random_deviations3d(nx, ny, nz, amp=2e-4, seed=21)
    o.set_populations(f0)
    g.set_populations(f0)
    o.step(100)
    g.step(100)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    assert vel_l2(ug, uo) < 1e-5
    if walls:
        Wo, Wg = o.get_wall_force(), g.get_wall_force()
        assert np.abs(Wg - Wo).max() <= 1e-4 * np.abs(Wo).max()


def test_rest_state():
    # at rest with neutrally buoyant spheres: nothing moves, bitwise (every frame constant
    # and short sum of them is exact in FP32)
    sp = inputs3d.spheres([[10.0, 10.0, 12.0], [30.0, 10.0, 12.0]], [4.0, 5.0], [1.0, 1.0])
    wr = inputs3d.Workload3D(name="rest", nx=48, ny=20, nz=24, tau=0.7, nsteps=1,
                             g=(0.0, 0.0, -1e-5), **sp)
    g = gpu3(wr)
    g.step(50)
    assert not g.get_populations().any()
    x, u, w = g.get_particles()
    assert np.array_equal(x, wr.pos) and not u.any() and not w.any()


def test_full_size_suspension_one_step():
    """256^3 with 400 spheres, in the launch configuration the benchmark times: one step
    from a random state, every population checked against the oracle."""
    wl = inputs3d.suspension3d()
    log_case(f"3d full size {wl.name}, 1 step")
    f0 = inputs3d.random_deviations3d(wl.nx, wl.ny, wl.nz, amp=1e-4, seed=9).astype(np.float32)
    f0 = f0.astype(np.float64)  # exactly representable on the GPU
    rng = np.random.Generator(np.random.PCG64(10))
    wl.vel = rng.uniform(-0.01, 0.01, wl.vel.shape)
    wl.omega = rng.uniform(-1e-3, 1e-3, wl.omega.shape)
    g = gpu3(wl)
    g.set_populations(f0)
    g.step(1)
    fg = g.get_populations()
    Fg, Tg = g.get_particle_forces()
    xg, _, _ = g.get_particles()
    g.close()
    o = oracle3(wl)
    o.set_populations(f0)
    del f0
    o.step(1)
    fo = o.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    del fg, fo
    assert err <= STEP_TOL, err
    Fo, To = o.get_particle_forces()
    xo, _, _ = o.get_particles()
    assert np.abs(Fg - Fo).max() <= 1e-4 * np.abs(Fo).max()
    assert np.abs(Tg - To).max() <= 1e-4 * np.abs(To).max()
    assert np.abs(xg - xo).max() < 1e-9


@pytest.mark.parametrize("cap,nx", [(1, 48), (2, 48), (2, 200)])
def test_lists_filled_to_capacity_match_oracle(cap, nx):
    """Lists exactly as long as the spheres need: with capacity 1 every entry sits in the
    tiles' heads; with 2, shared tiles hold the second entry in the list array (64 x 4 x 1
    tiles at nx = 48, whole rows at nx = 200)."""
    pos = [[20.0, 10.0, 8.0]] if cap == 1 else [[16.0, 10.0, 8.0], [30.0, 11.0, 9.0]]
    vel = [[0.01, 0.0, 0.004]] if cap == 1 else [[0.01, 0.0, 0.0], [-0.005, 0.004, 0.0]]
    sp = inputs3d.spheres(pos, [4.0] * len(pos), [1.3] * len(pos), vel=vel)
    wl = inputs3d.Workload3D(name="cap_exact", nx=nx, ny=20, nz=16, tau=0.7, nsteps=100,
                             G=(1e-5, 0.0, 0.0), **sp)
    log_case(f"3d lists filled to capacity {cap}, nx={nx}, 100 steps")
    g = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, list_capacity=cap))
    g.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    o = oracle3(wl)
    g.step(100)
    o.step(100)
    _, *ug = g.get_fields()
    _, *uo = o.get_fields()
    assert vel_l2(ug, uo) < 1e-5
    xg, _, _ = g.get_particles()
    xo, _, _ = o.get_particles()
    assert np.abs(xg - xo).max() < 1e-4
    g.close()


def test_list_overflow_and_instability_poison_the_handle():
    sp = inputs3d.spheres([[10.0, 6.0, 6.0], [12.0, 6.0, 6.0]], [4.0, 4.0], [1.2, 1.2])
    wl = inputs3d.Workload3D(name="cap", nx=32, ny=12, nz=12, tau=0.8, nsteps=1, **sp)
    log_case("3d list overflow")
    g = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, list_capacity=1))
    # two spheres share tiles but each list holds one: the binning flags it
    with pytest.raises(dilbm.DilbmError) as e:
        g.set_particles(wl.pos, wl.radius, wl.density)
    assert e.value.status == dilbm.ECAPACITY
    assert g.step_status(1) == dilbm.ESTATE
    g.close()
    log_case("3d instability")
    w2 = inputs3d.Workload3D(name="unstable", nx=16, ny=8, nz=8, tau=0.8, nsteps=1)
    g = gpu3(w2)
    f = np.zeros((19, 8, 8, 16))
    f[1] = 2.0  # a strong +x stream: rho = 3, u = 2/3 > 0.5
    g.set_populations(f)
    assert g.step_status(1) == dilbm.EUNSTABLE
    assert g.step_status(1) == dilbm.ESTATE
    g.get_fields()  # reads still work
    g.close()


def test_spheres_set_after_fluid_steps():
    """Spheres set on a solve that has been stepping without them (whole-row tiles): the
    sphere buffers are laid out anew under the same populations."""
    rng = np.random.Generator(np.random.PCG64(31))
    dims = (256, 12, 10)
    sp = inputs3d.random_spheres(rng, dims, 4, rmin=2.5, rmax=4.0, speed=0.01)
    wl = inputs3d.Workload3D(name="late", nx=256, ny=12, nz=10, tau=0.75, nsteps=1,
                             G=(1e-5, 0.0, 0.0))
    log_case("3d spheres set after 30 fluid steps, 256x12x10")
    o = oracle3(wl)
    g = gpu3(wl)
    o.step(30)
    g.step(30)
    o.set_particles(sp["pos"], sp["radius"], sp["density"], sp["vel"], sp["omega"])
    g.set_particles(sp["pos"], sp["radius"], sp["density"], sp["vel"], sp["omega"])
    o.step(30)
    g.step(30)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    assert vel_l2(ug, uo) < 1e-5
    xo, _, _ = o.get_particles()
    xg, _, _ = g.get_particles()
    assert np.abs(xg - xo).max() < 1e-6


def test_populations_round_trip_mid_run():
    """Populations read out and written back after some steps (the stored frame of a
    nonzero step count) continue exactly as an uninterrupted run (no spheres: the run is
    deterministic)."""
    wl = inputs3d.Workload3D(name="trip", nx=200, ny=12, nz=10, tau=0.7, nsteps=1,
                             G=(2e-5, -1e-5, 5e-6), wall_mask=inputs3d.WALL_Z, wall_h=2.0)
    f0 = inputs3d.random_deviations3d(wl.nx, wl.ny, wl.nz, amp=2e-4, seed=33)
    log_case("3d populations round trip at step 37")
    a = gpu3(wl)
    a.set_populations(f0)
    a.step(60)
    b = gpu3(wl)
    b.set_populations(f0)
    b.step(37)
    b.set_populations(b.get_populations())
    b.step(23)
    assert np.array_equal(a.get_populations(), b.get_populations())
    a.close()
    b.close()


def test_failure_stops_a_long_call_within_two_chunks():
    """Uniform acceleration G = 1e-3 drives |u| past 0.5 at step 500: a call of 4000 steps
    stops within two 32-step chunks of the failure and returns the error."""
    wl = inputs3d.Workload3D(name="blowup", nx=48, ny=16, nz=12, tau=0.8, nsteps=1,
                             G=(1e-3, 0.0, 0.0))
    log_case("3d blow-up in a long call")
    g = gpu3(wl)
    assert g.step_status(4000) == dilbm.EUNSTABLE
    n = g.step_count()
    assert 500 < n <= 501 + 2 * 32, n
    assert g.step_status(1) == dilbm.ESTATE
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_tile_lists_follow_a_fast_sphere(q):
    """Tile lists kept across steps and rebuilt once a sphere has moved half their skin: a
    sphere driven at a prescribed 0.25 lattice units per step crosses 50 units in 200 steps
    (a rebuild every few steps) past a free sphere, against the oracle."""
    sp = inputs3d.spheres([[16.0, 16.0, 12.0], [50.0, 18.0, 26.0]], [5.0, 4.0], [1.5, 1.2],
                          vel=[[0.25, 0.04, 0.02], [0.0, 0.0, 0.0]], fixed=[1, 0])
    wl = inputs3d.Workload3D(name="fast", nx=96, ny=32, nz=40, tau=0.8, nsteps=200, **sp)
    log_case(f"3d tile lists follow a fast sphere, D3Q{q}")
    o = o3.Oracle3Solver(o3.Oracle3Params(
        nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, rho0=wl.rho0, eps=wl.eps, cutoff=wl.cutoff,
        G=tuple(wl.G), g=tuple(wl.g), xi=wl.xi, lattice=q))
    o.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    g = gpu3(wl, lattice=q)
    o.step(200)
    g.step(200)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = vel_l2(ug, uo)
    print(f"3d fast sphere D3Q{q}: u rel L2 {e:.3e}")
    assert e < 1e-5
    xo, _, _ = o.get_particles()
    xg, _, _ = g.get_particles()
    d = np.abs(xg - xo)
    d = np.minimum(d, np.array([wl.nx, wl.ny, wl.nz]) - d)
    assert d.max() < 1e-4
    g.close()
