"""Pins of the oracle's body update inside the full step (Eqs. (22)-(24), (28), (29)).

In the first step from a fluid at rest (f = w rho0, G = 0) every node has u* = 0 and rho =
rho0, so the hydrodynamic force and torque of Eqs. (18)-(19) have closed forms: zero on a
body at rest, and for a moving body F = -rho0 sum_n phi_n u_s(x_n), T = -rho0 sum_n
phi_n (r_n x u_s(x_n)), with phi from Eq. (14) summed here directly.  What the step then
does with them is fixed by the paper's equations and the readings of the body update:
m = rho_s pi R^2, I = m R^2 / 2 (a disc of unit depth), forward Euler in velocity and
spin, trapezoidal in position, dt = 1.  Each test states the expected state after one
step from those formulas alone, so a mistake in the wiring (a wrong mass or inertia, a
flipped or attractive pair force, the wrong image or wall, a partner's radius or density
taken for the body's own) fails at least one of them; tests/test_oracle_mutants.py
checks that on planted copies of the oracle.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")

EPS_P, EPS_P1, EPS_W, EPS_W1, XI = 1.0e4, 2.0e4, 5.0e3, 7.0e3, 1.0


def _solver(nx, ny, pos, radius, density, vel=None, omega=None, walls=0, h=3.0, g=(0.0, 0.0),
            eps=2.0):
    import oracle

    p = oracle.OracleParams(nx=nx, ny=ny, tau=0.7, rho0=1.0, eps=eps, cutoff=4.0, G=(0.0, 0.0),
                            g=g, wall_mask=walls, wall_h=h, eps_p=EPS_P, eps_p1=EPS_P1,
                            eps_w=EPS_W, eps_w1=EPS_W1, xi=XI)
    s = oracle.OracleSolver(p)
    n = len(radius)
    s.set_particles(np.asarray(pos, float), np.asarray(radius, float),
                    np.asarray(density, float),
                    None if vel is None else np.asarray(vel, float),
                    None if omega is None else np.asarray(omega, float), np.zeros(n, np.uint8))
    return s


def _mass(R, rho_s):
    return rho_s * math.pi * R * R


def _pair_force_eq28(d_vec, ri, rj):
    """Eq. (28) as printed: the force on body i from body j, d_vec = X_i - X_j."""
    d = math.hypot(*d_vec)
    if d > ri + rj + XI:
        return np.zeros(2)
    if d <= ri + rj:
        return np.asarray(d_vec) * (ri + rj - d) / EPS_P1
    return np.asarray(d_vec) * (ri + rj + XI - d) ** 2 / EPS_P


def _wall_force_eq29(d_vec, r):
    """Eq. (29) as printed: d_vec = X_i - X_i', the image across the wall surface."""
    d = math.hypot(*d_vec)
    if d > 2 * r + XI:
        return np.zeros(2)
    if d <= 2 * r:
        return np.asarray(d_vec) * (2 * r - d) / EPS_W1
    return np.asarray(d_vec) * (2 * r + XI - d) ** 2 / EPS_W


def _expect_after_one_step(x0, u0, w0, F, T, R, rho_s):
    m = _mass(R, rho_s)
    inertia = 0.5 * m * R * R
    u1 = np.asarray(u0, float) + np.asarray(F, float) / m
    w1 = w0 + T / inertia
    x1 = np.asarray(x0, float) + 0.5 * (np.asarray(u0, float) + u1)
    return x1, u1, w1


@pytest.mark.parametrize("branch", ["soft", "overlap"])
def test_pair_repulsion_moves_both_discs_apart(branch):
    """Two discs at rest, one across the periodic seam from the other (minimum image),
    different radii and densities: after one step U_i = F_28 / m_i, X_i += U_i / 2, and the
    two momenta cancel."""
    nx, ny = 64, 48
    Ra, Rb = 5.0, 3.5
    rho_a, rho_b = 1.3, 2.1
    e = np.array([0.8, 0.6])
    d = Ra + Rb + (0.4 if branch == "soft" else -0.3)
    xa = np.array([60.2, 20.0])
    xb = xa + e * d  # x beyond nx: wrapped by the solver
    xb_wrapped = np.array([xb[0] - nx, xb[1]])
    s = _solver(nx, ny, [xa, xb_wrapped], [Ra, Rb], [rho_a, rho_b])
    s.step(1)
    x, u, w = s.get_particles()
    F, T = s.get_particle_forces()
    assert np.all(F == 0.0) and np.all(T == 0.0)  # fluid at rest, bodies at rest
    fa = _pair_force_eq28(xa - xb, Ra, Rb)
    assert np.dot(fa, xa - xb) > 0  # repulsive (pins the direction of the test formula)
    xa1, ua1, _ = _expect_after_one_step(xa, (0, 0), 0.0, fa, 0.0, Ra, rho_a)
    xb1, ub1, _ = _expect_after_one_step(xb_wrapped, (0, 0), 0.0, -fa, 0.0, Rb, rho_b)
    assert np.allclose(u[0], ua1, rtol=1e-12, atol=0)
    assert np.allclose(u[1], ub1, rtol=1e-12, atol=0)
    assert np.allclose(x[0], xa1, rtol=0, atol=1e-12)
    assert np.allclose(x[1], xb1, rtol=0, atol=1e-12)
    assert np.allclose(_mass(Ra, rho_a) * u[0] + _mass(Rb, rho_b) * u[1], 0.0, atol=1e-16)
    assert np.all(w == 0.0)


def test_pair_beyond_reach_does_not_move():
    nx, ny = 64, 48
    xa = np.array([20.0, 20.0])
    xb = xa + np.array([5.0 + 3.5 + XI + 1e-6, 0.0])
    s = _solver(nx, ny, [xa, xb], [5.0, 3.5], [1.3, 2.1])
    s.step(1)
    x, u, w = s.get_particles()
    assert np.all(u == 0.0) and np.all(w == 0.0)
    assert np.array_equal(x, np.array([xa, xb]))


def test_wall_repulsion_uses_the_image_across_the_nearer_surface():
    """Walls on both seams (surfaces at h and N - h).  Four discs, each within Eq. (29)'s
    reach of one surface only: the bottom and left ones in the soft zone, the top and right
    ones overlapping their image.  After one step U = F_29 / m, pointing away from the
    wall."""
    nx, ny, h = 64, 48, 3.0
    R = np.array([4.0, 4.0, 3.0, 3.5])
    rho = np.array([1.5, 1.2, 1.8, 1.1])
    pos = np.array([
        [20.0, h + R[0] + 0.25],          # bottom, 2 delta = 2R + 0.5: soft zone
        [44.0, ny - h - (R[1] - 0.2)],    # top, 2 delta = 2R - 0.4: overlap
        [h + R[2] + 0.3, 24.0],           # left, soft zone
        [nx - h - (R[3] - 0.1), 30.0],    # right, overlap
    ])
    s = _solver(nx, ny, pos, R, rho, walls=3, h=h)
    s.step(1)
    x, u, w = s.get_particles()
    F, T = s.get_particle_forces()
    assert np.all(F == 0.0) and np.all(T == 0.0)
    images = [
        np.array([0.0, 2 * (pos[0, 1] - h)]),
        np.array([0.0, -2 * ((ny - h) - pos[1, 1])]),
        np.array([2 * (pos[2, 0] - h), 0.0]),
        np.array([-2 * ((nx - h) - pos[3, 0]), 0.0]),
    ]
    away = [np.array([0, 1]), np.array([0, -1]), np.array([1, 0]), np.array([-1, 0])]
    for b in range(4):
        f = _wall_force_eq29(images[b], R[b])
        assert np.dot(f, away[b]) > 0
        xb1, ub1, _ = _expect_after_one_step(pos[b], (0, 0), 0.0, f, 0.0, R[b], rho[b])
        assert np.allclose(u[b], ub1, rtol=1e-12, atol=0), b
        assert np.allclose(x[b], xb1, rtol=0, atol=1e-12), b
        assert w[b] == 0.0


def _rigid_body_force_torque(nx, ny, X, R, U, omega, eps=2.0, cutoff=4.0, rho0=1.0):
    """Eqs. (14), (18), (19) at u* = 0, rho = rho0, one body: F = -rho0 sum phi u_s,
    T = -rho0 sum phi (r x u_s), u_s = U + omega x r, summed over every node."""
    i = np.arange(nx) + 0.5
    j = np.arange(ny) + 0.5
    rx = (i[None, :] - X[0] + nx / 2) % nx - nx / 2
    ry = (j[:, None] - X[1] + ny / 2) % ny - ny / 2
    rx, ry = np.broadcast_arrays(rx, ry)
    l = R - np.hypot(rx, ry)
    phi = np.where(l >= -cutoff * eps, 0.5 * (1.0 + np.tanh(2.0 * l / eps)), 0.0)
    usx = U[0] - omega * ry
    usy = U[1] + omega * rx
    F = -rho0 * np.array([(phi * usx).sum(), (phi * usy).sum()])
    T = -rho0 * (phi * (rx * usy - ry * usx)).sum()
    return F, T


@pytest.mark.parametrize("U,omega", [((0.0, 0.0), 2e-3), ((3e-3, -1e-3), 0.0),
                                     ((2e-3, 1.5e-3), -1e-3)])
def test_moving_disc_in_fluid_at_rest(U, omega):
    """A free disc moving and spinning in a fluid at rest, away from everything: the first
    step's hydrodynamic force and torque are the closed forms above, and the disc ends the
    step with U + F/m, omega + T/(m R^2 / 2) and X + (U_0 + U_1)/2."""
    nx, ny = 48, 40
    X = np.array([20.3, 17.6])
    R, rho_s = 6.0, 1.4
    s = _solver(nx, ny, [X], [R], [rho_s], vel=[U], omega=[omega])
    s.step(1)
    x, u, w = s.get_particles()
    F, T = s.get_particle_forces()
    Fe, Te = _rigid_body_force_torque(nx, ny, X, R, np.array(U), omega)
    scale = max(np.abs(Fe).max(), 1e-300)
    assert np.allclose(F[0], Fe, rtol=1e-11, atol=1e-12 * scale)
    assert T[0] == pytest.approx(Te, rel=1e-11, abs=1e-14)
    x1, u1, w1 = _expect_after_one_step(X, U, omega, Fe, Te, R, rho_s)
    assert np.allclose(u[0] - np.array(U), u1 - np.array(U), rtol=1e-10, atol=1e-18)
    assert (w[0] - omega) == pytest.approx(w1 - omega, rel=1e-10, abs=1e-18)
    assert np.allclose(x[0], x1, rtol=0, atol=1e-12)
    if omega != 0.0:
        # the torque opposes the spin (the fluid at rest brakes it)
        assert Te * omega < 0 and abs(w[0]) < abs(omega)


def test_heavy_disc_buoyancy_factor():
    """Gravity alone (Eq. (22) with rho_f = rho0): a heavy and a light disc at rest start
    with U = (rho0/rho_s - 1) g in one step, in opposite directions.  As Eqs. (22) and (27)
    are printed, g points away from the direction in which a heavy body sinks."""
    nx, ny = 64, 48
    g = (0.0, -2e-5)
    pos = [[16.0, 24.0], [48.0, 24.0]]
    R = [5.0, 4.0]
    rho = [1.5, 0.8]
    s = _solver(nx, ny, pos, R, rho, g=g)
    s.step(1)
    x, u, w = s.get_particles()
    for b in range(2):
        ue = (1.0 / rho[b] - 1.0) * np.array(g)
        assert np.allclose(u[b], ue, rtol=1e-13, atol=0)
        assert np.allclose(x[b], np.array(pos[b]) + 0.5 * ue, rtol=0, atol=1e-13)
    assert np.dot(u[0], g) < 0 < np.dot(u[1], g)
