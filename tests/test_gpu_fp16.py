"""GPU parity of FP16 population storage against the FP64 oracle, for the one-node-per-lane
tiles and the 512 x 1 tiles that hold two neighbouring nodes per lane (tile shape 5).

Tolerances, fixed before measuring.  One step from the same state: the GPU starts from the
FP16 copy of the input (round to nearest, 2^-11 of each value) and stores its result in
FP16 with stochastic rounding (under one FP16 ulp, 2^-10 of the value), with FP32
arithmetic in between; so every population is within 2^-8 of the largest deviation, and
forces (sums of rho (u_s - u*) built from the rounded inputs) within 5e-3 of the largest.
Many steps: the stated FP16 bounds, velocity relative L2 <= 2e-3, positions <= 1e-2.
"""
import numpy as np
import pytest

from paper_2106_08950_amd import dilbm, inputs
from helpers import gpu_solver, log_case, oracle_solver, velocity_rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

STEP_TOL16 = 2.0**-8
F16 = dilbm.STORE_FP16


def _random_case(seed, nx, ny, nb, walls=0, overlap=True, amp=1e-3):
    rng = np.random.default_rng(seed)
    b = inputs.random_bodies(rng, nx, ny, nb, rmin=3.0, rmax=9.0, allow_overlap=overlap,
                             fixed_frac=0.3)
    wl = inputs.Workload(name=f"f16rand{seed}", nx=nx, ny=ny, tau=float(rng.uniform(0.55, 1.4)),
                         nsteps=1, eps=float(rng.uniform(1.0, 2.5)), G=(2e-5, -1e-5),
                         g=(0.0, 1e-5), wall_mask=walls, wall_h=3.0, **b)
    f0 = inputs.random_deviations(nx, ny, amp=amp, seed=seed)
    return wl, f0


CASES16 = [
    # seed, nx, ny, bodies, walls (even nx: tile shape 5 needs it)
    (41, 16, 16, 3, 0),
    (42, 78, 45, 6, 3),     # ragged: the second 512-node tile of no row exists, rows of 78
    (43, 1030, 37, 14, 1),  # two 512-node tiles and a ragged third per row
    (44, 600, 70, 9, 2),    # x walls: supports across the periodic x seam
]


@pytest.mark.parametrize("seed,nx,ny,nb,walls", CASES16)
@pytest.mark.parametrize("tile", [0, 5])
def test_fp16_one_step_matches_oracle(seed, nx, ny, nb, walls, tile):
    wl, f0 = _random_case(seed, nx, ny, nb, walls)
    log_case(f"FP16 one step seed={seed} {nx}x{ny} walls={walls} tile={tile}")
    o = oracle_solver(wl)
    o.set_populations(f0)
    o.step(1)
    g = gpu_solver(wl, storage=F16, tile=tile)
    g.set_populations(f0)
    g.step(1)
    fo, fg = o.get_populations(), g.get_populations()
    scale = np.abs(fo).max()
    err = np.abs(fg - fo).max() / scale
    assert err <= STEP_TOL16, err
    Fo, To = o.get_particle_forces()
    Fg, Tg = g.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 5e-3 * max(np.abs(Fo).max(), 1e-30)
    assert np.abs(Tg - To).max() <= 5e-3 * max(np.abs(To).max(), 1e-30)
    if walls:
        Wo, Wg = o.get_wall_force(), g.get_wall_force()
        assert np.abs(Wg - Wo).max() <= 5e-3 * np.abs(Wo).max()
    _, uxo, uyo = o.get_fields()
    _, uxg, uyg = g.get_fields()
    assert velocity_rel_l2(uxg, uyg, uxo, uyo) < 2e-3
    g.close()


@pytest.mark.parametrize("seed,nx,ny,walls", [(51, 96, 64, 0), (52, 1100, 40, 3)])
def test_fp16_pair_tiles_many_steps(seed, nx, ny, walls):
    wl, f0 = _random_case(seed, nx, ny, 8, walls, overlap=False, amp=2e-4)
    log_case(f"FP16 300 steps, tile 5, seed={seed} {nx}x{ny} walls={walls}")
    o = oracle_solver(wl)
    o.set_populations(f0)
    g = gpu_solver(wl, storage=F16, tile=5)
    g.set_populations(f0)
    o.step(300)
    g.step(300)
    _, uxo, uyo = o.get_fields()
    _, uxg, uyg = g.get_fields()
    e = velocity_rel_l2(uxg, uyg, uxo, uyo)
    assert e < 2e-3, e
    xo, _, _ = o.get_particles()
    xg, _, _ = g.get_particles()
    d = np.abs(xg - xo)
    d = np.minimum(d, [nx, ny] - d)
    assert d.max() < 1e-2
    g.close()


@pytest.mark.parametrize("tile", [0, 5])
def test_fp16_rest_stays_at_rest_bitwise(tile):
    wl = inputs.cylinder_channel()
    wl = inputs.Workload(**{**wl.__dict__, "G": (0.0, 0.0), "g": (0.0, -1e-3)})
    wl.pos = np.array([[100.0, 40.0], [40.0, 30.0]])
    wl.radius = np.array([10.0, 6.0])
    wl.density = np.array([1.0, 1.0])
    wl.vel = np.zeros((2, 2))
    wl.omega = np.zeros(2)
    wl.fixed = np.array([1, 0], np.uint8)
    log_case(f"FP16 rest, tile {tile}")
    g = gpu_solver(wl, storage=F16, tile=tile)
    g.step(200)
    assert np.all(g.get_populations() == 0.0)
    g.close()


@pytest.mark.parametrize("case", [(31, 70, 40, 0, 0, 0, 1), (33, 64, 33, 0, 1, 0, 0),
                                  (34, 130, 20, 1, 1, 0, 1)])
def test_fp16_pair_tiles_open_ends_one_step(case):
    from test_gpu_boundaries import _bcase

    wl, f0 = _bcase(*case)
    log_case(f"FP16 open ends one step {case} tile 5")
    o = oracle_solver(wl)
    o.set_populations(f0)
    o.step(1)
    g = gpu_solver(wl, storage=F16, tile=5)
    g.set_populations(f0)
    g.step(1)
    fo, fg = o.get_populations(), g.get_populations()
    assert np.abs(fg - fo).max() / np.abs(fo).max() <= STEP_TOL16
    _, uxo, uyo = o.get_fields()
    _, uxg, uyg = g.get_fields()
    assert velocity_rel_l2(uxg, uyg, uxo, uyo) < 2e-3
    g.close()


def test_fp16_pair_tiles_inflow_cylinder():
    from test_gpu_boundaries import _inflow_cylinder

    wl = _inflow_cylinder()
    log_case(f"FP16 inflow cylinder, tile 5, {wl.nsteps} steps")
    o = oracle_solver(wl)
    o.step(wl.nsteps)
    g = gpu_solver(wl, storage=F16, tile=5)
    g.step(wl.nsteps)
    _, uxo, uyo = o.get_fields()
    _, uxg, uyg = g.get_fields()
    e = velocity_rel_l2(uxg, uyg, uxo, uyo)
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    ef = abs(Fg[0, 0] - Fo[0, 0]) / abs(Fo[0, 0])
    print(f"inflow cylinder FP16 tile 5: u rel L2 {e:.3e}, drag rel error {ef:.3e}")
    assert e < 2e-3 and ef < 2e-2
    g.close()


def test_automatic_scale_is_ten_on_d2q9():
    """The automatic FP16 scale (the default) stores exactly as an explicit k = 10: the
    same populations, bit for bit, after 10 steps of a driven flow from a random state (on
    256 x 256 some values lie where 2^9 or 2^11 would move them into or out of FP16's
    subnormals)."""
    from oracle import binding as o2  # noqa: F401  (the fixture builds it)
    log_case("fp16 automatic scale vs 2^10")
    f0 = inputs.random_deviations(256, 256, amp=1e-4, seed=21)
    out = []
    for k in (dilbm.FP16_SCALE_AUTO, 10):
        with dilbm.Solver(dilbm.Params(nx=256, ny=256, tau=0.7, body_force=(1e-5, 2e-6),
                                       storage=F16, fp16_scale_log2=k)) as s:
            s.set_populations(f0)
            s.step(10)
            out.append(s.get_populations())
    assert np.array_equal(out[0], out[1])


def test_automatic_scale_keeps_a_dense_fast_state_finite():
    """A uniform state of rho = 3.5 moving at 0.45 along x (inside what a step accepts):
    its axis population S (f_1 - w_1) = 4 (3.5 h - 1) with h = 1 + 1.35 + 0.91125 - 0.30375
    is 37.4, which FP16 holds at 2^10 (38 300) but not at 2^11 (76 600 > 65 504).  The
    automatic scale keeps it exactly uniform; k = 11 stores an infinity and the step
    reports the state unstable."""
    from oracle import binding as o2

    nx, ny, rho, u = 64, 32, 3.5, 0.45
    w = o2.lattice()[2]
    f = (o2.feq(rho, u, 0.0) - w)[:, None, None] * np.ones((1, ny, nx))
    log_case("fp16 dense fast uniform state, automatic scale and 2^11")
    with dilbm.Solver(dilbm.Params(nx=nx, ny=ny, tau=0.8, storage=F16)) as s:
        s.set_populations(f)
        s.step(20)
        r, ux, uy = s.get_fields()
    np.testing.assert_allclose(r, rho, rtol=1e-2)
    np.testing.assert_allclose(ux, u, rtol=1e-2)
    assert np.abs(uy).max() < 1e-2
    with dilbm.Solver(dilbm.Params(nx=nx, ny=ny, tau=0.8, storage=F16,
                                   fp16_scale_log2=11)) as s:
        s.set_populations(f)
        assert s.step_status(1) == dilbm.EUNSTABLE
