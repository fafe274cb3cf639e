"""Pins of the three-dimensional oracle's open ends in x (non-equilibrium extrapolation,
Guo, Zheng & Shi 2002; the treatment the paper gives its physical boundaries in
Section 3), against what the mathematics fixes:

* the boundary node's mass and momentum: the equilibrium part carries the boundary state
  exactly, the extrapolated non-equilibrium part carries no mass and the momentum
  -(1 - 1/tau) G/2 (the neighbour's velocity includes half the body force);
* a neighbour at equilibrium hands the boundary node exactly the equilibrium of the
  boundary state;
* exact reduction to the pinned two-dimensional oracle's open channel on a z-uniform
  problem (D3Q19 and D3Q27 project onto D2Q9 there), for a parabolic velocity inlet with
  a density outlet and for a density inlet with a zero-gradient outlet;
* the duct profile is the product of the channel profiles across y and across z;
* invalid open-end parameters are refused.
"""
import numpy as np
import pytest

from oracle import binding as o2
from oracle import binding3d as o3

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _moments(q, f_dev, rho0):
    cx, cy, cz, w, _ = o3.lattice(q)
    f = f_dev + w * rho0
    return f.sum(), np.array([(cx * f).sum(), (cy * f).sum(), (cz * f).sum()])


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("kind", ["velocity", "density", "zero_gradient"])
def test_boundary_node_mass_and_momentum(q, kind):
    rng = np.random.default_rng(q + len(kind))
    tau, rho0 = 0.83, 1.0
    G = np.array([3e-5, -1e-5, 2e-5])
    u_nb_eq = rng.uniform(-0.05, 0.05, 3)
    f_nb = o3.feq(1.01, u_nb_eq, q) + rng.normal(0.0, 1e-3, q) - o3.lattice(q)[3] * rho0
    rho_nb, j_nb = _moments(q, f_nb, rho0)
    u_nb = (j_nb + 0.5 * G) / rho_nb
    u_set = np.array([0.04, 0.01, -0.02])
    if kind == "velocity":
        fp, rb, ub = o3.nee_node(tau, rho0, f_nb, G, rho_set=None, u_set=u_set, q=q)
        want_rho, want_u = rho_nb, u_set
    elif kind == "density":
        fp, rb, ub = o3.nee_node(tau, rho0, f_nb, G, rho_set=0.997, u_set=None, q=q)
        want_rho, want_u = 0.997, u_nb
    else:
        fp, rb, ub = o3.nee_node(tau, rho0, f_nb, G, q=q)
        want_rho, want_u = rho_nb, u_nb
    assert rb == pytest.approx(want_rho, rel=1e-15) and np.allclose(ub, want_u, rtol=0, atol=1e-16)
    rho_b, j_b = _moments(q, fp, rho0)
    assert rho_b == pytest.approx(want_rho, rel=1e-14)
    np.testing.assert_allclose(j_b, want_rho * want_u - (1.0 - 1.0 / tau) * 0.5 * G,
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("q", [19, 27])
def test_neighbour_at_equilibrium_gives_the_boundary_equilibrium(q):
    rho0 = 1.0
    w = o3.lattice(q)[3]
    f_nb = o3.feq(1.003, [0.02, -0.01, 0.005], q) - w * rho0
    u_b = np.array([0.05, 0.0, 0.01])
    fp, rb, _ = o3.nee_node(0.7, rho0, f_nb, u_set=u_b, q=q)
    np.testing.assert_allclose(fp + w * rho0, o3.feq(rb, u_b, q), rtol=0, atol=1e-16)
    assert rb == pytest.approx(1.003, rel=1e-15)


def _pair(q, inlet_kind, outlet_kind, nz=3, steps=150):
    nx, ny, h, tau = 36, 18, 3.0, 0.8
    common = dict(tau=tau, wall_mask=1, wall_h=h, x_boundary=1, inlet_kind=inlet_kind,
                  outlet_kind=outlet_kind, rho_in=1.002, rho_out=0.999)
    p3 = o3.Oracle3Params(nx=nx, ny=ny, nz=nz, G=(2e-6, 0.0, 0.0), inlet_profile=1,
                          u_in=(0.03, 0.0, 0.0), lattice=q, **common)
    p2 = o2.OracleParams(nx=nx, ny=ny, G=(2e-6, 0.0), inlet_profile=1, u_in=(0.03, 0.0),
                         **common)
    s3, s2 = o3.Oracle3Solver(p3), o2.OracleSolver(p2)
    s3.step(steps)
    s2.step(steps)
    return s3.get_fields(), s2.get_fields()


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("kinds", [(0, 0), (1, 1)])
def test_z_uniform_open_channel_is_the_two_dimensional_one(q, kinds):
    (rho3, ux3, uy3, uz3), (rho2, ux2, uy2) = _pair(q, *kinds)
    assert np.abs(ux2).max() > 1e-3  # the flow is established
    assert not uz3.any()
    for k in range(rho3.shape[0]):
        np.testing.assert_allclose(rho3[k], rho2, rtol=0, atol=1e-13)
        np.testing.assert_allclose(ux3[k], ux2, rtol=0, atol=1e-13)
        np.testing.assert_allclose(uy3[k], uy2, rtol=0, atol=1e-13)


def test_duct_profile_is_the_product_of_the_channel_profiles():
    ny, nz, h = 20, 14, 3.0
    duct = o3.Oracle3Params(nx=10, ny=ny, nz=nz, tau=0.8, wall_mask=1 | 4, wall_h=h,
                            x_boundary=1, inlet_profile=2, u_in=(0.02, 0.0, 0.0))
    across_y = o3.Oracle3Params(nx=10, ny=ny, nz=nz, tau=0.8, wall_mask=1, wall_h=h,
                                x_boundary=1, inlet_profile=1)
    across_z = o3.Oracle3Params(nx=10, ny=nz, nz=ny, tau=0.8, wall_mask=1, wall_h=h,
                                x_boundary=1, inlet_profile=1)
    vals = np.array([[o3.inlet_shape(duct, j, k) for k in range(nz)] for j in range(ny)])
    for j in range(ny):
        for k in range(nz):
            assert vals[j, k] == pytest.approx(
                o3.inlet_shape(across_y, j, 0) * o3.inlet_shape(across_z, k, 0), rel=1e-15)
    assert vals.max() <= 1.0 and vals[0].max() == 0.0 and vals[:, 0].max() == 0.0
    np.testing.assert_allclose(vals, vals[::-1, ::-1], rtol=0, atol=1e-15)  # symmetric
    assert o3.inlet_shape(o3.Oracle3Params(nx=10, ny=ny, nz=nz, tau=0.8, x_boundary=1), 5, 5) == 1.0


@pytest.mark.parametrize("bad", [dict(nx=2), dict(wall_mask=2), dict(inlet_kind=2),
                                 dict(outlet_kind=3), dict(inlet_profile=3),
                                 dict(inlet_kind=1, rho_in=0.0), dict(rho_out=-1.0),
                                 dict(x_boundary=2)])
def test_invalid_open_ends_are_refused(bad):
    kw = dict(nx=12, ny=8, nz=6, tau=0.8, x_boundary=1)
    kw.update(bad)
    with pytest.raises(o3.Oracle3Error):
        o3.Oracle3Solver(o3.Oracle3Params(**kw))
