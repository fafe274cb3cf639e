"""Pins of the oracle's pointwise operators against what the paper and the mathematics fix.

Each test checks an operator against a closed form or identity that is independent of
the formula the oracle codes: a dropped term, a wrong sign, a wrong weight or a
transposed operand breaks at least one of them.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _ora():
    import oracle

    return oracle


def test_velocities_follow_eq3_trig_form():
    # Eq. (3): c_0 = 0; c_i = (cos, sin)((i-1) pi/2) for i=1..4;
    # c_i = sqrt(2) (cos, sin)((2i-1) pi/4) for i=5..8.
    cx, cy, w, cs2 = _ora().lattice()
    exp = [(0.0, 0.0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        exp.append((math.cos(a), math.sin(a)))
    for i in range(5, 9):
        a = (2 * i - 1) * math.pi / 4
        exp.append((math.sqrt(2) * math.cos(a), math.sqrt(2) * math.sin(a)))
    exp = np.round(np.array(exp)).astype(int)
    assert np.array_equal(cx, exp[:, 0])
    assert np.array_equal(cy, exp[:, 1])


def test_weights_eq4_and_lattice_isotropy():
    cx, cy, w, cs2 = _ora().lattice()
    assert w[0] == pytest.approx(4 / 9, abs=0)
    assert np.allclose(w[1:5], 1 / 9, rtol=0, atol=1e-17)
    assert np.allclose(w[5:], 1 / 36, rtol=0, atol=1e-17)
    c = np.stack([cx, cy], 1).astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    # second moment: cs^2 I with cs^2 = 1/3 (the value the appendix's equilibrium moments need)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), cs2 * np.eye(2), atol=1e-16)
    assert cs2 == pytest.approx(1 / 3, rel=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    d = np.eye(2)
    iso = cs2**2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                    + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments_appendix(seed):
    # appendix: sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = cs^2 rho I + rho u u
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 2)
    cx, cy, w, cs2 = _ora().lattice()
    c = np.stack([cx, cy], 1).astype(float)
    f = _ora().feq(rho, u[0], u[1])
    assert abs(f.sum() - rho) < 1e-15
    assert np.allclose(c.T @ f, rho * u, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", f, c, c),
                       cs2 * rho * np.eye(2) + rho * np.outer(u, u), atol=1e-15)
    # third moment of the second-order equilibrium: cs^2 rho (u_a d_bc + u_b d_ac + u_c d_ab)
    d = np.eye(2)
    m3 = cs2 * rho * (np.einsum("a,bc->abc", u, d) + np.einsum("b,ac->abc", u, d)
                      + np.einsum("c,ab->abc", u, d))
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", f, c, c, c), m3, atol=1e-15)


def test_phi_eq14_profile():
    phi = _ora().phi
    eps = 2.0
    assert phi(0.0, eps) == 0.5
    for l in np.linspace(-7.9, 7.9, 41):
        # (1 + tanh z)/2 = 1/(1 + exp(-2z)) with z = 2l/eps (logistic form)
        assert phi(l, eps) == pytest.approx(1.0 / (1.0 + math.exp(-4 * l / eps)), rel=1e-14)
        assert phi(l, eps) + phi(-l, eps) == pytest.approx(1.0, abs=1e-15)
    ls = np.linspace(-8, 8, 200)
    vals = [phi(l, eps) for l in ls]
    assert all(b >= a for a, b in zip(vals, vals[1:]))
    # support cut-off at l = -4 eps: phi is about 1.1e-7 just inside and exactly 0 beyond
    assert phi(-8.0, eps) == pytest.approx(0.5 * (1 - math.tanh(8.0)), rel=1e-12)
    assert 1.0e-7 < phi(-8.0, eps) < 1.2e-7
    assert phi(-8.0 - 1e-9, eps) == 0.0
    assert phi(-100.0, eps) == 0.0
    assert phi(100.0, eps) == 1.0
    # interface thickness: phi goes from 0.119 to 0.881 over l in [-eps/2, eps/2]
    assert phi(eps / 2, eps) == pytest.approx((1 + math.tanh(1.0)) / 2, rel=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_force_term_eq15_moments_and_equilibrium_form(seed):
    o = _ora()
    rng = np.random.default_rng(100 + seed)
    tau = rng.uniform(0.51, 2.0)
    rho = rng.uniform(0.8, 1.2)
    us = rng.uniform(-0.1, 0.1, 2)
    ust = rng.uniform(-0.1, 0.1, 2)
    cx, cy, w, cs2 = o.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    F = o.force_term(tau, rho, us, ust)
    k = 1 - 1 / (2 * tau)
    tol = 1e-14 * np.abs(F).max()
    assert abs(F.sum()) < tol
    assert np.allclose(c.T @ F, k * rho * (us - ust), rtol=0, atol=tol)
    assert np.allclose(np.einsum("i,ia,ib->ab", F, c, c),
                       k * rho * (np.outer(us, us) - np.outer(ust, ust)), rtol=0, atol=tol)
    # Eq. (15) replaces B[f^eq(rho,u_s) - f^eq(rho,u)] of Eq. (12): it equals
    # (1 - 1/2tau)[f^eq(rho, u_s) - f^eq(rho, u*)] exactly for the second-order f^eq.
    alt = k * (o.feq(rho, *us) - o.feq(rho, *ust))
    assert np.allclose(F, alt, rtol=0, atol=tol)
    # no solid-fluid slip, no force
    assert np.allclose(o.force_term(tau, rho, us, us), 0, atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_body_force_term_moments(seed):
    o = _ora()
    rng = np.random.default_rng(200 + seed)
    tau = rng.uniform(0.51, 2.0)
    u = rng.uniform(-0.1, 0.1, 2)
    G = rng.uniform(-1e-3, 1e-3, 2)
    cx, cy, w, cs2 = o.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    Gi = o.guo_term(tau, u, G)
    k = 1 - 1 / (2 * tau)
    tol = 1e-14 * np.abs(Gi).max()
    assert abs(Gi.sum()) < tol
    assert np.allclose(c.T @ Gi, k * G, rtol=0, atol=tol)
    assert np.allclose(np.einsum("i,ia,ib->ab", Gi, c, c),
                       k * (np.outer(u, G) + np.outer(G, u)), rtol=0, atol=tol)


def _rand_f(rng, amp=5e-3):
    return rng.uniform(-amp, amp, 9)


@pytest.mark.parametrize("seed", range(6))
def test_collide_node_fluid_only_conserves(seed):
    o = _ora()
    rng = np.random.default_rng(300 + seed)
    tau = rng.uniform(0.51, 2.0)
    G = rng.uniform(-1e-4, 1e-4, 2)
    fd = _rand_f(rng)
    cx, cy, w, cs2 = o.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    st, fp, rho, u, ust, fb = o.collide_node(tau, 1.0, fd, G=G)
    assert st == 0
    f = fd + w
    fps = fp + w
    assert abs(fps.sum() - f.sum()) < 1e-15
    assert np.allclose(c.T @ fps - c.T @ f, G, atol=1e-16)
    # velocity carries half the body force: rho u = sum c f + G/2
    assert np.allclose(rho * u, c.T @ f + G / 2, atol=1e-16)
    # with G = 0 the non-equilibrium part relaxes by (1 - 1/tau): Eq. (1)
    st, fp0, rho0_, u0, _, _ = o.collide_node(tau, 1.0, fd)
    feq = o.feq(rho0_, *u0)
    assert np.allclose(fp0 + w - feq, (1 - 1 / tau) * (f - feq), atol=1e-16)


@pytest.mark.parametrize("seed", range(8))
def test_collide_node_with_bodies_momentum_balance(seed):
    o = _ora()
    rng = np.random.default_rng(400 + seed)
    tau = rng.uniform(0.51, 2.0)
    G = rng.uniform(-1e-4, 1e-4, 2)
    nb = int(rng.integers(1, 4))
    phis = rng.uniform(0.05, 1.0, nb)  # sums above 1 exercise the weighting
    us = rng.uniform(-0.05, 0.05, (nb, 2))
    fd = _rand_f(rng)
    cx, cy, w, cs2 = o.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    st, fp, rho, u, ust, fb = o.collide_node(tau, 1.0, fd, phis, us, G)
    assert st == 0
    f = fd + w
    fps = fp + w
    S = phis.sum()
    wb = phis * min(1.0, 1.0 / S)
    assert abs(fps.sum() - f.sum()) < 1e-15
    # momentum gained = G + sum_b w_b rho (u_s,b - u*) = G - sum_b (force on body b)
    gain = c.T @ fps - c.T @ f
    expect = G + (wb[:, None] * rho * (us - ust[None, :])).sum(0)
    assert np.allclose(gain, expect, atol=1e-16)
    assert np.allclose(gain, G - fb.sum(0), atol=1e-16)
    # appendix (non-equilibrium first moment) with the body-force half step:
    # sum c (f - f^eq(rho, u)) = -1/2 sum_b w_b rho (u_s,b - u*) - G/2
    feq = o.feq(rho, *u)
    assert np.allclose(c.T @ (f - feq),
                       -0.5 * (wb[:, None] * rho * (us - ust[None, :])).sum(0) - G / 2,
                       atol=1e-16)
    # the literal Eq. (18) scale is (1 - 1/2tau) times the momentum-exchange force
    st1, fp1, *_rest, fb1 = o.collide_node(tau, 1.0, fd, phis, us, G, force_mode=1)
    assert np.array_equal(fp1, fp)
    assert np.allclose(fb1, (1 - 1 / (2 * tau)) * fb, atol=1e-18)


@pytest.mark.parametrize("seed", range(4))
def test_full_solid_node_takes_body_velocity(seed):
    # phi = 1, no body force: the post-collision momentum is rho u_s
    o = _ora()
    rng = np.random.default_rng(500 + seed)
    tau = rng.uniform(0.51, 2.0)
    us = rng.uniform(-0.05, 0.05, 2)
    fd = _rand_f(rng)
    cx, cy, w, cs2 = o.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    st, fp, rho, u, ust, fb = o.collide_node(tau, 1.0, fd, [1.0], [us])
    assert np.allclose(c.T @ (fp + w), rho * us, atol=1e-16)
    # corrected velocity is half way between u* and u_s
    assert np.allclose(u, 0.5 * (ust + us), atol=1e-17)


def test_collide_node_flags_instability():
    o = _ora()
    fd = np.zeros(9)
    fd[1] = 2.0  # rho = 3, |u| = 2/3 > 0.5
    st, *_ = o.collide_node(0.8, 1.0, fd)
    assert st == -4
    fd = np.full(9, -0.2)  # rho < 0
    st, *_ = o.collide_node(0.8, 1.0, fd)
    assert st == -4


def test_particle_particle_repulsion_eq28():
    o = _ora()
    ri, rj, xi, ep, ep1 = 5.0, 3.0, 1.0, 1.0e4, 2.0e4
    e = np.array([0.6, 0.8])  # unit direction X_i - X_j
    # beyond the threshold
    assert np.all(o.pp_force(e * (ri + rj + xi + 1e-9), ri, rj, xi, ep, ep1) == 0)
    # soft zone: (1/eps_P)(X_i - X_j)(r_i + r_j + xi - d)^2
    d = ri + rj + 0.25
    assert np.allclose(o.pp_force(e * d, ri, rj, xi, ep, ep1), e * d * 0.75**2 / ep, rtol=1e-14)
    # overlap: (1/eps_P')(X_i - X_j)(r_i + r_j - d)
    d = ri + rj - 0.5
    assert np.allclose(o.pp_force(e * d, ri, rj, xi, ep, ep1), e * d * 0.5 / ep1, rtol=1e-14)
    # at contact the overlap branch gives zero; just outside the soft branch gives xi^2/eps_P
    assert np.all(o.pp_force(e * (ri + rj), ri, rj, xi, ep, ep1) == 0)
    f = o.pp_force(e * (ri + rj + 1e-12), ri, rj, xi, ep, ep1)
    assert np.allclose(f, e * (ri + rj) * xi**2 / ep, rtol=1e-9)
    # repulsive: along X_i - X_j
    assert np.dot(o.pp_force(e * (ri + rj + 0.5), ri, rj, xi, ep, ep1), e) > 0


def test_particle_wall_repulsion_eq29():
    o = _ora()
    r, xi, ew, ew1 = 4.0, 1.0, 5.0e3, 6.0e3
    e = np.array([0.0, 1.0])
    assert np.all(o.pw_force(e * (2 * r + xi + 1e-9), r, xi, ew, ew1) == 0)
    d = 2 * r + 0.5
    assert np.allclose(o.pw_force(e * d, r, xi, ew, ew1), e * d * 0.25 / ew, rtol=1e-14)
    d = 2 * r - 0.25
    assert np.allclose(o.pw_force(e * d, r, xi, ew, ew1), e * d * 0.25 / ew1, rtol=1e-14)


def test_newton_euler_update_constant_force_closed_form():
    # Eqs. (22)-(24) with forward-Euler velocity and trapezoidal position: exact for a
    # constant force: U = U0 + F t/m, X = X0 + U0 t + F t^2/(2m), omega = omega0 + T t/I
    o = _ora()
    m, I = 3.7, 11.3
    F = np.array([1.3e-3, -2.1e-3])
    T = 4.0e-4
    x = np.array([10.0, 20.0])
    u = np.array([0.01, -0.02])
    om = 1e-3
    x0, u0, om0 = x.copy(), u.copy(), om
    for t in range(1, 201):
        x, u, om = o.body_update(m, I, F, T, x, u, om)
    t = 200
    assert np.allclose(u, u0 + F * t / m, rtol=1e-13, atol=1e-17)
    assert np.allclose(x, x0 + u0 * t + F * t * t / (2 * m), rtol=1e-13)
    assert om == pytest.approx(om0 + T * t / I, rel=1e-13)
