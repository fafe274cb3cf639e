"""GPU parity of the open inlet / outlet columns (non-equilibrium extrapolation, the paper's
treatment of its physical boundaries) against the FP64 oracle: one step from random states
for every kind of inlet and outlet and several tile shapes, a fixed cylinder in an inflow
channel over many steps in FP32 and FP16, and a uniform stream that must stay as it is.
Tolerances are those of the periodic cases (one step: 256 * 2^-24 of the largest
deviation; many steps: the stated velocity relative L2)."""
import numpy as np
import pytest

from paper_2106_08950_amd import inputs
from helpers import gpu_solver, log_case, oracle_solver, velocity_rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

U32 = 2.0**-24
STEP_TOL = 256 * U32
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])

BCASES = [
    # seed, nx, ny, walls, inlet_kind, inlet_profile, outlet_kind
    (31, 70, 40, 0, 0, 0, 1),    # uniform velocity inlet, zero-gradient outlet
    (32, 77, 45, 1, 0, 1, 0),    # parabolic velocity inlet between y walls, pressure outlet
    (33, 64, 33, 0, 1, 0, 0),    # pressure inlet, pressure outlet
    (34, 130, 20, 1, 1, 0, 1),   # pressure inlet, zero-gradient outlet, y walls
]


def _bodies_inside(rng, nx, ny, n, margin):
    """n discs whose supports stay clear of the two outermost columns on each side."""
    pos, rad = inputs.place_discs(rng, nx - 2 * margin, ny, n, lambda r: r.uniform(2.5, 4.5))
    pos = pos + np.array([margin, 0.0])
    return inputs._bodies(pos, rad, np.full(len(rad), 1.3))


def _bcase(seed, nx, ny, walls, ik, prof, ok):
    rng = np.random.default_rng(seed)
    eps = float(rng.uniform(1.0, 2.0))
    b = _bodies_inside(rng, nx, ny, 3, margin=int(4 * eps + 4.5 + 3))
    wl = inputs.Workload(name=f"open{seed}", nx=nx, ny=ny, tau=float(rng.uniform(0.6, 1.3)),
                         nsteps=1, eps=eps, G=(1e-5, -2e-6), g=(0.0, 1e-5), wall_mask=walls,
                         wall_h=3.0, x_boundary=1, inlet_kind=ik, inlet_profile=prof,
                         outlet_kind=ok, u_in=(0.04, 0.003), rho_in=1.002, rho_out=0.999, **b)
    f0 = inputs.random_deviations(nx, ny, amp=1e-3, seed=seed)
    return wl, f0


@pytest.mark.parametrize("case", BCASES)
@pytest.mark.parametrize("tile", [0, 2, 3])
def test_one_step_with_open_ends_matches_oracle(case, tile):
    wl, f0 = _bcase(*case)
    log_case(f"open ends one step {case} tile={tile}")
    o = oracle_solver(wl)
    o.set_populations(f0)
    o.step(1)
    g = gpu_solver(wl, tile=tile)
    g.set_populations(f0)
    g.step(1)
    fo, fg = o.get_populations(), g.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    assert err <= STEP_TOL, err
    ro, uxo, uyo = o.get_fields()
    rg, uxg, uyg = g.get_fields()
    assert np.abs(rg - ro).max() <= 1e-5 and velocity_rel_l2(uxg, uyg, uxo, uyo) < 1e-5
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 1e-4 * max(np.abs(Fo).max(), 1e-30)


def _inflow_cylinder(storage_steps=400):
    # the Section 3.1 set-up in small: a fixed cylinder in a uniform stream entering at the
    # inlet column and leaving through a zero-gradient outlet, periodic across
    return inputs.Workload(name="inflow_cylinder", nx=160, ny=64, tau=0.8,
                           nsteps=storage_steps, eps=2.0, x_boundary=1, inlet_kind=0,
                           outlet_kind=1, u_in=(0.04, 0.0),
                           **inputs._bodies([[48.0, 32.3]], [6.0], [1.0], fixed=[1]))


@pytest.mark.parametrize("storage,tol", [(0, 1e-5), (1, 2e-3)])
def test_inflow_cylinder_matches_oracle(storage, tol):
    wl = _inflow_cylinder()
    log_case(f"inflow cylinder 160x64, {wl.nsteps} steps, storage={storage}")
    o = oracle_solver(wl)
    o.step(wl.nsteps)
    g = gpu_solver(wl, storage=storage)
    g.step(wl.nsteps)
    _, uxo, uyo = o.get_fields()
    _, uxg, uyg = g.get_fields()
    e = velocity_rel_l2(uxg, uyg, uxo, uyo)
    Fo, _ = o.get_particle_forces()
    Fg, _ = g.get_particle_forces()
    ef = abs(Fg[0, 0] - Fo[0, 0]) / abs(Fo[0, 0])
    print(f"inflow cylinder storage={storage}: u rel L2 {e:.3e}, drag rel error {ef:.3e}")
    assert e < tol and ef < 10 * tol
    assert np.abs(uxo[:, 0] - 0.04).max() < 1e-14            # the oracle's inlet holds u_in
    assert np.abs(uxg[:, 0] - 0.04).max() < 1e-6 * (1 if storage == 0 else 1e3)


def test_uniform_stream_stays_put_on_gpu():
    u = 0.05
    wl = inputs.Workload(name="stream", nx=96, ny=24, tau=0.7, nsteps=300, x_boundary=1,
                         inlet_kind=0, outlet_kind=1, u_in=(u, 0.0))
    cu = CX * u
    feq = W * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u * u) - W
    f0 = np.broadcast_to(feq[:, None, None], (9, wl.ny, wl.nx)).copy()
    log_case("uniform stream through inlet and outlet")
    g = gpu_solver(wl)
    g.set_populations(f0)
    g.step(wl.nsteps)
    rho, ux, uy = g.get_fields()
    assert np.abs(ux - u).max() < 1e-6 and np.abs(uy).max() < 1e-6
    assert np.abs(rho - 1.0).max() < 1e-6
