"""Pins of the oracle's open inlet / outlet columns: non-equilibrium extrapolation (Guo,
Zheng & Shi 2002), the scheme the paper applies to its physical boundaries (Section 3).

Checked against what the scheme and the lattice fix rather than against its own formula:
the moments the boundary node must carry (mass and momentum of the boundary state; the
stress of that equilibrium plus the relaxed non-equilibrium stress of the neighbour, the
latter computed here independently), a uniform stream that must be a fixed point, and
plane Poiseuille flow fed through a parabolic velocity inlet and a pressure outlet between
halfway bounce-back walls, whose profile and pressure gradient have closed forms."""
import math

import numpy as np
import pytest

from oracle import binding as B

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _eq(rho, u):
    """Second-order D2Q9 equilibrium written out from its moments (textbook form)."""
    cu = CX * u[0] + CY * u[1]
    return W * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u[0] ** 2 + u[1] ** 2))


def _neighbour(seed, rho0=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-2e-3, 2e-3, 9) + _eq(1.0, (0.03, -0.01)) - W * rho0


@pytest.mark.parametrize("seed", range(4))
def test_velocity_inlet_node_carries_the_boundary_state(seed):
    rho0, tau = 1.0, 0.8
    fn = _neighbour(seed)
    ub = (0.04, 0.005)
    out, rb, u = B.nee_node(tau, rho0, fn, u_set=ub)
    f = out + W * rho0
    rho_nb = (fn + W * rho0).sum()
    assert rb == pytest.approx(rho_nb, rel=1e-15)          # density from the neighbour
    assert f.sum() == pytest.approx(rho_nb, rel=1e-14)     # mass of the boundary state
    assert np.allclose([(CX * f).sum(), (CY * f).sum()], rho_nb * np.array(ub),
                       rtol=0, atol=1e-15)                 # momentum rho_b u_b (G = 0)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.3])
def test_boundary_stress_is_equilibrium_plus_relaxed_neighbour_stress(tau):
    rho0 = 1.0
    fn = _neighbour(7)
    fnf = fn + W * rho0
    rho_nb = fnf.sum()
    u_nb = np.array([(CX * fnf).sum(), (CY * fnf).sum()]) / rho_nb
    # the neighbour's non-equilibrium stress, from its own moments
    pi_neq = np.array([[(a * b * (fnf - _eq(rho_nb, u_nb))).sum() for b in (CX, CY)]
                       for a in (CX, CY)])
    ub = (0.02, 0.0)
    out, rb, _ = B.nee_node(tau, rho0, fn, u_set=ub)
    f = out + W * rho0
    pi = np.array([[(a * b * f).sum() for b in (CX, CY)] for a in (CX, CY)])
    pi_eq = np.array([[(a * b * _eq(rho_nb, ub)).sum() for b in (CX, CY)] for a in (CX, CY)])
    assert np.allclose(pi, pi_eq + (1 - 1 / tau) * pi_neq, rtol=0, atol=1e-15)


def test_pressure_node_with_neighbour_at_equilibrium_is_that_equilibrium():
    rho0 = 1.0
    u = (0.03, 0.01)
    fn = _eq(1.004, u) - W * rho0
    out, rb, ub = B.nee_node(0.9, rho0, fn, rho_set=0.998)
    assert rb == 0.998 and np.allclose(ub, u, atol=1e-15)
    assert np.allclose(out + W * rho0, _eq(0.998, u), rtol=0, atol=1e-15)


def test_uniform_stream_through_inlet_and_outlet_is_a_fixed_point():
    u = (0.05, 0.0)
    p = B.OracleParams(nx=40, ny=12, tau=0.7, x_boundary=1, inlet_kind=0, outlet_kind=1,
                       u_in=u)
    f0 = np.broadcast_to((_eq(1.0, u) - W)[:, None, None], (9, 12, 40)).copy()
    with B.OracleSolver(p) as s:
        s.set_populations(f0)
        s.step(200)
        f = s.get_populations()
        rho, ux, uy = s.get_fields()
    assert np.abs(f - f0).max() < 1e-14
    assert np.abs(ux - u[0]).max() < 1e-14 and np.abs(rho - 1.0).max() < 1e-14


def test_poiseuille_through_velocity_inlet_and_pressure_outlet():
    # halfway bounce-back walls at y = 0 and y = H are exact for plane Poiseuille flow at
    # tau = 1/2 + sqrt(3/16); the parabolic inlet feeds the fully developed profile, so the
    # whole channel should carry it, with dp/dx = mu u'' = -8 rho0 nu U / H^2
    H, L, U = 16, 64, 1e-3
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    p = B.OracleParams(nx=L, ny=H, tau=tau, bb_walls_y=1, x_boundary=1, inlet_kind=0,
                       inlet_profile=1, outlet_kind=0, u_in=(U, 0.0), rho_out=1.0)
    with B.OracleSolver(p) as s:
        s.step(6000)
        rho, ux, uy = s.get_fields()
    y = np.arange(H) + 0.5
    shape = 4 * (y / H) * (1 - y / H)
    mid = ux[:, L // 2]
    assert np.abs(mid / mid.max() - shape / shape.max()).max() < 2e-3      # parabolic
    # mass flux rho u is the inlet's all along the channel
    flux = (rho * ux).sum(axis=0)
    assert np.abs(flux[1:-1] / (U * shape).sum() - flux[1] / (U * shape).sum()).max() < 1e-3
    assert np.abs(uy[:, 16:L - 8]).max() < 1e-4 * U    # developed: no cross flow
    assert np.abs(uy).max() < 5e-3 * U                  # entrance effect at the inlet column
    # pressure gradient: slope of rho along the channel centre, away from the ends
    xs = np.arange(8, L - 8)
    slope = np.polyfit(xs, rho[H // 2, 8:L - 8], 1)[0]
    assert slope == pytest.approx(-3 * 8 * nu * U / H ** 2, rel=2e-2)
    assert rho[:, -1] == pytest.approx(np.ones(H), abs=1e-12)              # outlet density


def test_neighbour_velocity_carries_half_the_body_force():
    # reading: the neighbour's velocity is the one its own collision uses, u = (j + G/2)/rho,
    # so its non-equilibrium part holds -G/2 of momentum and the boundary node carries
    # rho_b u_b - (1 - 1/tau) G/2
    rho0, tau, G = 1.0, 0.7, (3e-4, -2e-4)
    fn = _neighbour(11)
    ub = (0.02, 0.01)
    out, rb, _ = B.nee_node(tau, rho0, fn, G=G, u_set=ub)
    f = out + W * rho0
    mom = np.array([(CX * f).sum(), (CY * f).sum()])
    assert np.allclose(mom, rb * np.array(ub) - (1 - 1 / tau) * 0.5 * np.array(G),
                       rtol=0, atol=1e-15)
