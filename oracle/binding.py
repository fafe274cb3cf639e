"""ctypes binding of the FP64 oracle library (test infrastructure only).

Argument marshalling only: every number is computed in ``dilbm_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dilbm_oracle.c")
_LIB = os.path.join(_HERE, "libdilbm_oracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


def compile_c(src: str, lib: str, force: bool) -> str:
    """Compile one oracle source into a shared library with gcc (FP64, no FMA
    contraction, OpenMP)."""
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


def build_oracle(force: bool = True) -> str:
    """Compile ``libdilbm_oracle.so`` and the three-dimensional ``libdilbm3d_oracle.so``."""
    compile_c(os.path.join(_HERE, "dilbm3d_oracle.c"),
              os.path.join(_HERE, "libdilbm3d_oracle.so"), force)
    return compile_c(_SRC, _LIB, force)


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double), ("eps", C.c_double), ("cutoff", C.c_double),
        ("G", C.c_double * 2), ("g", C.c_double * 2),
        ("wall_mask", C.c_uint32), ("wall_h", C.c_double),
        ("force_mode", C.c_int32),
        ("eps_p", C.c_double), ("eps_p1", C.c_double), ("eps_w", C.c_double),
        ("eps_w1", C.c_double), ("xi", C.c_double),
        ("bb_walls_y", C.c_int32),
        ("x_boundary", C.c_int32), ("inlet_kind", C.c_int32), ("inlet_profile", C.c_int32),
        ("outlet_kind", C.c_int32), ("u_in", C.c_double * 2),
        ("rho_in", C.c_double), ("rho_out", C.c_double),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        # DILBM_ORACLE_LIB: a copy built elsewhere (the planted-mistake tests load
        # deliberately broken copies this way); the library here is built on demand
        path = os.environ.get("DILBM_ORACLE_LIB") or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build_oracle(force=False)
        lib = C.CDLL(path)
        lib.ora_lattice.argtypes = [_ip, _ip, _dp, _dp]
        lib.ora_feq.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        lib.ora_phi.argtypes = [C.c_double, C.c_double, C.c_double]
        lib.ora_phi.restype = C.c_double
        lib.ora_force_term.argtypes = [C.c_double] * 6 + [_dp]
        lib.ora_guo_term.argtypes = [C.c_double] * 5 + [_dp]
        lib.ora_collide_node.argtypes = [C.c_double, C.c_double, _dp, C.c_int32, _dp, _dp, _dp,
                                         C.c_double, C.c_double, C.c_int32, _dp, _dp, _dp, _dp,
                                         _dp]
        lib.ora_collide_node.restype = C.c_int32
        lib.ora_nee_node.argtypes = [C.c_double, C.c_double, _dp, C.c_double, C.c_double,
                                     C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_double,
                                     _dp, _dp, _dp]
        lib.ora_pp_force.argtypes = [C.c_double] * 7 + [_dp]
        lib.ora_pw_force.argtypes = [C.c_double] * 6 + [_dp]
        lib.ora_body_update.argtypes = [C.c_double] * 5 + [_dp] * 5
        lib.ora_create.argtypes = [C.POINTER(_Params), C.POINTER(C.c_void_p)]
        lib.ora_create.restype = C.c_int32
        lib.ora_destroy.argtypes = [C.c_void_p]
        lib.ora_set_particles.argtypes = [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp, _dp, _u8p]
        lib.ora_set_particles.restype = C.c_int32
        lib.ora_set_populations.argtypes = [C.c_void_p, _dp]
        lib.ora_set_populations.restype = C.c_int32
        lib.ora_get_populations.argtypes = [C.c_void_p, _dp]
        lib.ora_get_populations.restype = C.c_int32
        lib.ora_step.argtypes = [C.c_void_p, C.c_int64]
        lib.ora_step.restype = C.c_int32
        lib.ora_get_fields.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.ora_get_fields.restype = C.c_int32
        lib.ora_get_particle_forces.argtypes = [C.c_void_p, _dp, _dp]
        lib.ora_get_particle_forces.restype = C.c_int32
        lib.ora_get_particles.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.ora_get_particles.restype = C.c_int32
        lib.ora_get_wall_force.argtypes = [C.c_void_p, _dp]
        lib.ora_get_wall_force.restype = C.c_int32
        lib.ora_num_threads.restype = C.c_int32
        lib.ora_set_num_threads.argtypes = [C.c_int32]
        lib.ora_set_num_threads.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(_L().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's node loops (its results do not depend on the count)."""
    _L().ora_set_num_threads(int(n))


def lattice():
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9)
    cs2 = np.zeros(1)
    _L().ora_lattice(cx.ctypes.data_as(_ip), cy.ctypes.data_as(_ip), _ptr(w), _ptr(cs2))
    return cx, cy, w, float(cs2[0])


def feq(rho, ux, uy):
    out = np.zeros(9)
    _L().ora_feq(rho, ux, uy, _ptr(out))
    return out


def phi(l, eps, cutoff=4.0):
    return float(_L().ora_phi(l, eps, cutoff))


def force_term(tau, rho, us, ustar):
    out = np.zeros(9)
    _L().ora_force_term(tau, rho, us[0], us[1], ustar[0], ustar[1], _ptr(out))
    return out


def guo_term(tau, u, G):
    out = np.zeros(9)
    _L().ora_guo_term(tau, u[0], u[1], G[0], G[1], _ptr(out))
    return out


def collide_node(tau, rho0, f_dev, phis=(), us=(), G=(0.0, 0.0), force_mode=0):
    """One node, no streaming.  Returns (status, fpost_dev, rho, u, ustar, force_b)."""
    f_dev = _f64(f_dev)
    nb = len(phis)
    ph = _f64(np.asarray(phis, dtype=np.float64).reshape(-1))
    usa = np.asarray(us, dtype=np.float64).reshape(nb, 2) if nb else np.zeros((0, 2))
    usx = _f64(usa[:, 0].copy())
    usy = _f64(usa[:, 1].copy())
    fp = np.zeros(9)
    rho = np.zeros(1)
    u = np.zeros(2)
    ust = np.zeros(2)
    fb = np.zeros(max(nb, 1) * 2)
    st = _L().ora_collide_node(tau, rho0, _ptr(f_dev), nb, _ptr(ph) if nb else None,
                               _ptr(usx) if nb else None, _ptr(usy) if nb else None,
                               G[0], G[1], force_mode, _ptr(fp), _ptr(rho), _ptr(u), _ptr(ust),
                               _ptr(fb))
    return int(st), fp, float(rho[0]), u, ust, fb[: 2 * nb].reshape(nb, 2)


def nee_node(tau, rho0, f_nb_dev, G=(0.0, 0.0), rho_set=None, u_set=None):
    """Non-equilibrium extrapolation at one boundary node from its neighbour's populations:
    rho_set / u_set prescribe the boundary state, None takes the neighbour's.
    Returns (f*_b deviations, rho_b, u_b)."""
    fn = _f64(f_nb_dev)
    out = np.zeros(9)
    rb = C.c_double()
    ub = np.zeros(2)
    ux, uy = (0.0, 0.0) if u_set is None else u_set
    _L().ora_nee_node(tau, rho0, _ptr(fn), G[0], G[1], int(rho_set is None),
                      0.0 if rho_set is None else float(rho_set), int(u_set is None), ux, uy,
                      _ptr(out), C.byref(rb), _ptr(ub))
    return out, rb.value, ub


def pp_force(d, ri, rj, xi, eps_p, eps_p1):
    out = np.zeros(2)
    _L().ora_pp_force(d[0], d[1], ri, rj, xi, eps_p, eps_p1, _ptr(out))
    return out


def pw_force(d, r, xi, eps_w, eps_w1):
    out = np.zeros(2)
    _L().ora_pw_force(d[0], d[1], r, xi, eps_w, eps_w1, _ptr(out))
    return out


def body_update(m, I, F, T, x, u, om):
    xs = [C.c_double(x[0]), C.c_double(x[1]), C.c_double(u[0]), C.c_double(u[1]),
          C.c_double(om)]
    _L().ora_body_update(m, I, F[0], F[1], T, *[C.byref(v) for v in xs])
    return (np.array([xs[0].value, xs[1].value]), np.array([xs[2].value, xs[3].value]),
            xs[4].value)


@dataclass
class OracleParams:
    nx: int
    ny: int
    tau: float
    rho0: float = 1.0
    eps: float = 2.0
    cutoff: float = 4.0
    G: tuple = (0.0, 0.0)
    g: tuple = (0.0, 0.0)
    wall_mask: int = 0
    wall_h: float = 4.0
    force_mode: int = 0
    eps_p: float = 1.0e4
    eps_p1: float = 1.0e4
    eps_w: float = 0.5e4
    eps_w1: float = 0.5e4
    xi: float = 1.0
    bb_walls_y: int = 0
    x_boundary: int = 0        # 1: inlet column x = 0, outlet column x = nx - 1
    inlet_kind: int = 0        # 0 velocity, 1 pressure
    inlet_profile: int = 0     # 0 uniform, 1 parabolic across the channel
    outlet_kind: int = 0       # 0 pressure, 1 zero gradient
    u_in: tuple = (0.0, 0.0)
    rho_in: float = 1.0
    rho_out: float = 1.0

    def _c(self):
        p = _Params()
        p.nx, p.ny = int(self.nx), int(self.ny)
        p.tau, p.rho0, p.eps, p.cutoff = self.tau, self.rho0, self.eps, self.cutoff
        p.G[0], p.G[1] = self.G
        p.g[0], p.g[1] = self.g
        p.wall_mask = int(self.wall_mask)
        p.wall_h = self.wall_h
        p.force_mode = int(self.force_mode)
        p.eps_p, p.eps_p1, p.eps_w, p.eps_w1, p.xi = (self.eps_p, self.eps_p1, self.eps_w,
                                                      self.eps_w1, self.xi)
        p.bb_walls_y = int(self.bb_walls_y)
        p.x_boundary, p.inlet_kind = int(self.x_boundary), int(self.inlet_kind)
        p.inlet_profile, p.outlet_kind = int(self.inlet_profile), int(self.outlet_kind)
        p.u_in[0], p.u_in[1] = self.u_in
        p.rho_in, p.rho_out = self.rho_in, self.rho_out
        return p


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


class OracleSolver:
    """FP64 DI-LBM solver.  Populations are deviations f_i - w_i rho0, shape [9, ny, nx]."""

    def __init__(self, params: OracleParams):
        self.params = params
        h = C.c_void_p()
        cp = params._c()
        st = _L().ora_create(C.byref(cp), C.byref(h))
        if st != 0:
            raise OracleError(st, "ora_create")
        self._h = h
        self.nb = 0

    def close(self):
        if getattr(self, "_h", None):
            _L().ora_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what):
        if st != 0:
            raise OracleError(st, what)

    def set_particles(self, pos, radius, density, vel=None, omega=None, fixed=None):
        pos = _f64(pos, (-1, 2))
        n = pos.shape[0]
        radius = _f64(radius, (n,))
        density = _f64(density, (n,))
        vel = _f64(vel, (n, 2)) if vel is not None else None
        omega = _f64(omega, (n,)) if omega is not None else None
        fx = (np.ascontiguousarray(fixed, dtype=np.uint8).reshape(n)
              if fixed is not None else None)
        st = _L().ora_set_particles(self._h, n, _ptr(pos), _ptr(vel), _ptr(omega), _ptr(radius),
                                    _ptr(density),
                                    fx.ctypes.data_as(_u8p) if fx is not None else None)
        self._check(st, "ora_set_particles")
        self.nb = n

    def set_populations(self, f_dev):
        p = self.params
        f_dev = _f64(f_dev, (9, p.ny, p.nx))
        self._check(_L().ora_set_populations(self._h, _ptr(f_dev)), "ora_set_populations")

    def get_populations(self):
        p = self.params
        out = np.zeros((9, p.ny, p.nx))
        self._check(_L().ora_get_populations(self._h, _ptr(out)), "ora_get_populations")
        return out

    def step(self, n=1):
        self._check(_L().ora_step(self._h, int(n)), "ora_step")

    def step_status(self, n=1):
        return int(_L().ora_step(self._h, int(n)))

    def get_fields(self):
        p = self.params
        rho = np.zeros((p.ny, p.nx))
        ux = np.zeros((p.ny, p.nx))
        uy = np.zeros((p.ny, p.nx))
        self._check(_L().ora_get_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy)),
                    "ora_get_fields")
        return rho, ux, uy

    def get_particle_forces(self):
        f = np.zeros((max(self.nb, 1), 2))
        t = np.zeros(max(self.nb, 1))
        self._check(_L().ora_get_particle_forces(self._h, _ptr(f), _ptr(t)),
                    "ora_get_particle_forces")
        return f[: self.nb], t[: self.nb]

    def get_particles(self):
        x = np.zeros((max(self.nb, 1), 2))
        u = np.zeros((max(self.nb, 1), 2))
        w = np.zeros(max(self.nb, 1))
        self._check(_L().ora_get_particles(self._h, _ptr(x), _ptr(u), _ptr(w)),
                    "ora_get_particles")
        return x[: self.nb], u[: self.nb], w[: self.nb]

    def get_wall_force(self):
        f = np.zeros(2)
        self._check(_L().ora_get_wall_force(self._h, _ptr(f)), "ora_get_wall_force")
        return f
