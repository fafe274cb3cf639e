"""GPU parity of FP16 population storage on the three-dimensional path (D3Q19 and D3Q27)
against the FP64 3-D oracle on the same lattice, through the C ABI.

Tolerances, fixed before measuring, as for FP16 in two dimensions: one step from the same
state, every population within 2^-8 of the largest deviation and sphere forces and
torques within 5e-3 of the largest (the GPU starts from the FP16 copy of the input and
stores its result with stochastic rounding, under one FP16 ulp); many steps, velocity
relative L2 <= 2e-3 and positions <= 1e-2 lattice units (the stated FP16 bounds).
"""
import numpy as np
import pytest

from oracle import binding3d as o3
from paper_2106_08950_amd import dilbm, dilbm3d, inputs3d
from helpers import log_case, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

STEP_TOL16 = 2.0**-8
F16 = dilbm.STORE_FP16


def oracle3q(wl, q):
    s = o3.Oracle3Solver(o3.Oracle3Params(
        nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, rho0=wl.rho0, eps=wl.eps, cutoff=wl.cutoff,
        G=tuple(wl.G), g=tuple(wl.g), wall_mask=wl.wall_mask, wall_h=wl.wall_h,
        force_mode=wl.force_mode, eps_p=wl.eps_p, eps_p1=wl.eps_p1, eps_w=wl.eps_w,
        eps_w1=wl.eps_w1, xi=wl.xi, lattice=q))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def gpu16(wl, q):
    s = dilbm3d.Solver3D(dilbm3d.params_from_workload(wl, lattice=q, storage=F16))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def _case(seed, dims, nsph, walls, q, overlap=True, amp=1e-3, rmax=6.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    sp = inputs3d.random_spheres(rng, dims, nsph, rmin=2.5, rmax=rmax, speed=0.02, spin=2e-3,
                                 allow_overlap=overlap, fixed_frac=0.25)
    wl = inputs3d.Workload3D(name=f"f16case{seed}", nx=nx, ny=ny, nz=nz,
                             tau=0.55 + 0.1 * (seed % 5), nsteps=1, G=(1e-5, -4e-6, 2e-6),
                             g=(0.0, 0.0, -2e-5), wall_mask=walls, wall_h=3.0, **sp)
    f0 = np.random.Generator(np.random.PCG64(seed + 100)).uniform(-amp, amp,
                                                                  size=(q, nz, ny, nx))
    return wl, f0


CASES = [
    (1, (16, 16, 16), 3, 0),
    (2, (70, 9, 5), 4, inputs3d.WALL_Y),       # ragged in x and y
    (4, (64, 8, 12), 5, 7),                    # walls on every axis
    (7, (200, 6, 5), 4, inputs3d.WALL_Y),      # whole-row tiles, one partial
]


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("seed,dims,nsph,walls", CASES)
def test_fp16_3d_one_step_matches_oracle(seed, dims, nsph, walls, q):
    wl, f0 = _case(seed, dims, nsph, walls, q)
    log_case(f"3d FP16 one step D3Q{q} seed={seed} {dims} walls={walls}")
    o = oracle3q(wl, q)
    o.set_populations(f0)
    o.step(1)
    g = gpu16(wl, q)
    g.set_populations(f0)
    g.step(1)
    fo, fg = o.get_populations(), g.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    assert err <= STEP_TOL16, err
    Fo, To = o.get_particle_forces()
    Fg, Tg = g.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 5e-3 * max(np.abs(Fo).max(), 1e-30)
    assert np.abs(Tg - To).max() <= 5e-3 * max(np.abs(To).max(), 1e-30)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    assert rel_l2(np.stack(ug), np.stack(uo)) < 2e-3
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_fp16_3d_many_steps_match_oracle(q):
    wl, f0 = _case(11, (64, 40, 32), 6, 0, q, overlap=False, amp=2e-4, rmax=5.0)
    log_case(f"3d FP16 1000 steps D3Q{q}")
    o = oracle3q(wl, q)
    o.set_populations(f0)
    g = gpu16(wl, q)
    g.set_populations(f0)
    o.step(1000)
    g.step(1000)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    xo, _, _ = o.get_particles()
    xg, _, _ = g.get_particles()
    d = np.abs(xg - xo)
    d = np.minimum(d, np.array([wl.nx, wl.ny, wl.nz]) - d)
    print(f"3d FP16 D3Q{q} 1000 steps: u rel L2 {e:.3e}, position error {d.max():.3e}")
    assert e < 2e-3
    assert d.max() < 1e-2
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_fp16_3d_channel_with_fixed_sphere(q):
    wl = inputs3d.channel3d()
    log_case(f"3d FP16 channel D3Q{q}, 500 steps")
    o = oracle3q(wl, q)
    g = gpu16(wl, q)
    o.step(500)
    g.step(500)
    _, *uo = o.get_fields()
    _, *ug = g.get_fields()
    e = rel_l2(np.stack(ug), np.stack(uo))
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    ef = abs(Fg[0, 0] - Fo[0, 0]) / abs(Fo[0, 0])
    print(f"3d FP16 channel D3Q{q}: u rel L2 {e:.3e}, drag rel error {ef:.3e}")
    assert e < 2e-3 and ef < 2e-2
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_fp16_3d_rest_state_bitwise(q):
    sp = inputs3d.spheres([[10.0, 10.0, 12.0], [30.0, 10.0, 12.0]], [4.0, 5.0], [1.0, 1.0])
    wr = inputs3d.Workload3D(name="rest", nx=48, ny=20, nz=24, tau=0.7, nsteps=1,
                             g=(0.0, 0.0, -1e-5), **sp)
    log_case(f"3d FP16 rest D3Q{q}")
    g = gpu16(wr, q)
    g.step(50)
    assert not g.get_populations().any()
    x, u, w = g.get_particles()
    assert np.array_equal(x, wr.pos) and not u.any() and not w.any()
    g.close()


def test_fp16_3d_full_size_suspension_one_step():
    """256^3 with 400 spheres, FP16 on D3Q19, in the benchmark's launch configuration:
    one step from a random state, every population checked against the oracle."""
    wl = inputs3d.suspension3d()
    log_case(f"3d FP16 full size {wl.name}, 1 step")
    f0 = inputs3d.random_deviations3d(wl.nx, wl.ny, wl.nz, amp=1e-4, seed=29)
    g = gpu16(wl, 19)
    g.set_populations(f0)
    g.step(1)
    fg = g.get_populations()
    Fg, _ = g.get_particle_forces()
    g.close()
    o = oracle3q(wl, 19)
    o.set_populations(f0)
    del f0
    o.step(1)
    fo = o.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    del fg, fo
    assert err <= STEP_TOL16, err
    Fo, _ = o.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 5e-3 * np.abs(Fo).max()


@pytest.mark.parametrize("q,rho,k_over", [(27, 3.2, 9), (19, 3.5, 12)])
def test_automatic_scale_keeps_a_dense_fast_state_finite(q, rho, k_over):
    """A uniform state moving at 0.45 along x (inside what a step accepts) whose axis
    population S w_1 (rho h - 1), h = 1 + 1.35 + 0.91125 - 0.30375, FP16 holds at the
    automatic scale (2^8 on D3Q27: 16 (3.2 h - 1) = 135.4, times 256 is 34 700; 2^11 on
    D3Q19: 2 (3.5 h - 1) = 18.7, times 2048 is 38 300) but not at twice that (above
    65 504).  The automatic scale keeps it uniform; the larger k stores an infinity and
    the step reports the state unstable."""
    nx, ny, nz, u = 64, 16, 8, 0.45
    w = o3.lattice(q)[3]
    f = (o3.feq(rho, [u, 0.0, 0.0], q) - w)[:, None, None, None] * np.ones((1, nz, ny, nx))
    log_case(f"3d fp16 D3Q{q} dense fast uniform state, automatic scale and 2^{k_over}")
    with dilbm3d.Solver3D(dilbm3d.Params3D(nx=nx, ny=ny, nz=nz, tau=0.8, lattice=q,
                                           storage=F16)) as s:
        s.set_populations(f)
        s.step(20)
        r, ux, uy, uz = s.get_fields()
    np.testing.assert_allclose(r, rho, rtol=1e-2)
    np.testing.assert_allclose(ux, u, rtol=1e-2)
    assert max(np.abs(uy).max(), np.abs(uz).max()) < 1e-2
    with dilbm3d.Solver3D(dilbm3d.Params3D(nx=nx, ny=ny, nz=nz, tau=0.8, lattice=q,
                                           storage=F16, fp16_scale_log2=k_over)) as s:
        s.set_populations(f)
        assert s.step_status(1) == dilbm.EUNSTABLE
