"""Shared test helpers: build matching oracle and GPU solvers from one seeded workload."""
import numpy as np


def oracle_solver(wl, **kw):
    import oracle

    d = dict(nx=wl.nx, ny=wl.ny, tau=wl.tau, rho0=wl.rho0, eps=wl.eps, cutoff=wl.cutoff,
             G=tuple(wl.G), g=tuple(wl.g), wall_mask=wl.wall_mask, wall_h=wl.wall_h,
             force_mode=wl.force_mode, eps_p=wl.eps_p, eps_p1=wl.eps_p1, eps_w=wl.eps_w,
             eps_w1=wl.eps_w1, xi=wl.xi, x_boundary=wl.x_boundary, inlet_kind=wl.inlet_kind,
             inlet_profile=wl.inlet_profile, outlet_kind=wl.outlet_kind, u_in=tuple(wl.u_in),
             rho_in=wl.rho_in, rho_out=wl.rho_out)
    d.update(kw)
    s = oracle.OracleSolver(oracle.OracleParams(**d))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def gpu_solver(wl, **kw):
    from paper_2106_08950_amd import dilbm

    s = dilbm.Solver(dilbm.params_from_workload(wl, **kw))
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def velocity_rel_l2(ux, uy, ux_ref, uy_ref):
    return rel_l2(np.stack([ux, uy]), np.stack([ux_ref, uy_ref]))


def momentum(fdev):
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
    tot = fdev.reshape(9, -1).sum(axis=1)
    return np.array([cx @ tot, cy @ tot])


def log_case(msg):
    """Print and flush what a GPU step is about to run, so a fault names its case."""
    print(f"[gpu-case] {msg}", flush=True)
