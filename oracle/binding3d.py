"""ctypes binding of the three-dimensional FP64 oracle (D3Q19, spheres) -- test
infrastructure only.

Argument marshalling only: every number is computed in ``dilbm3d_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .binding import compile_c

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dilbm3d_oracle.c")
_LIB = os.path.join(_HERE, "libdilbm3d_oracle.so")
Q = 19

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double), ("eps", C.c_double), ("cutoff", C.c_double),
        ("G", C.c_double * 3), ("g", C.c_double * 3),
        ("wall_mask", C.c_uint32), ("wall_h", C.c_double),
        ("force_mode", C.c_int32),
        ("eps_p", C.c_double), ("eps_p1", C.c_double), ("eps_w", C.c_double),
        ("eps_w1", C.c_double), ("xi", C.c_double),
        ("lattice", C.c_int32),
        ("x_boundary", C.c_int32), ("inlet_kind", C.c_int32), ("inlet_profile", C.c_int32),
        ("outlet_kind", C.c_int32), ("u_in", C.c_double * 3), ("rho_in", C.c_double),
        ("rho_out", C.c_double),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        # DILBM_ORACLE3_LIB: a copy built elsewhere (planted-mistake tests)
        path = os.environ.get("DILBM_ORACLE3_LIB") or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            compile_c(_SRC, _LIB, force=False)
        lib = C.CDLL(path)
        lib.ora3_lattice.argtypes = [_ip, _ip, _ip, _dp, _dp]
        lib.ora3_feq.argtypes = [C.c_double, _dp, _dp]
        lib.ora3_force_term.argtypes = [C.c_double, C.c_double, _dp, _dp, _dp]
        lib.ora3_guo_term.argtypes = [C.c_double, _dp, _dp, _dp]
        lib.ora3_collide_node.argtypes = [C.c_double, C.c_double, _dp, C.c_int32, _dp, _dp, _dp,
                                          C.c_int32, _dp, _dp, _dp, _dp, _dp]
        lib.ora3_collide_node.restype = C.c_int32
        lib.ora3q_lattice.argtypes = [C.c_int32, _ip, _ip, _ip, _dp, _dp]
        lib.ora3q_feq.argtypes = [C.c_int32, C.c_double, _dp, _dp]
        lib.ora3q_force_term.argtypes = [C.c_int32, C.c_double, C.c_double, _dp, _dp, _dp]
        lib.ora3q_guo_term.argtypes = [C.c_int32, C.c_double, _dp, _dp, _dp]
        lib.ora3q_collide_node.argtypes = [C.c_int32] + lib.ora3_collide_node.argtypes
        lib.ora3q_collide_node.restype = C.c_int32
        lib.ora3q_nee_node.argtypes = [C.c_int32, C.c_double, C.c_double, _dp, _dp, C.c_int32,
                                       C.c_double, C.c_int32, _dp, _dp, _dp, _dp]
        lib.ora3_inlet_shape.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32]
        lib.ora3_inlet_shape.restype = C.c_double
        lib.ora3_pp_force.argtypes = [_dp] + [C.c_double] * 5 + [_dp]
        lib.ora3_pw_force.argtypes = [_dp] + [C.c_double] * 4 + [_dp]
        lib.ora3_body_update.argtypes = [C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp]
        lib.ora3_create.argtypes = [C.POINTER(_Params), C.POINTER(C.c_void_p)]
        lib.ora3_create.restype = C.c_int32
        lib.ora3_destroy.argtypes = [C.c_void_p]
        lib.ora3_set_particles.argtypes = [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp, _dp, _u8p]
        lib.ora3_set_particles.restype = C.c_int32
        for name in ("ora3_set_populations", "ora3_get_populations", "ora3_get_wall_force"):
            getattr(lib, name).argtypes = [C.c_void_p, _dp]
            getattr(lib, name).restype = C.c_int32
        lib.ora3_step.argtypes = [C.c_void_p, C.c_int64]
        lib.ora3_step.restype = C.c_int32
        lib.ora3_get_fields.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        lib.ora3_get_fields.restype = C.c_int32
        lib.ora3_get_particle_forces.argtypes = [C.c_void_p, _dp, _dp]
        lib.ora3_get_particle_forces.restype = C.c_int32
        lib.ora3_get_particles.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.ora3_get_particles.restype = C.c_int32
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def lattice(q=Q):
    """Velocities and weights of D3Q19 (q = 19) or D3Q27 (q = 27), and c_s^2."""
    cx, cy, cz = (np.zeros(q, np.int32) for _ in range(3))
    w = np.zeros(q)
    cs2 = np.zeros(1)
    _L().ora3q_lattice(q, cx.ctypes.data_as(_ip), cy.ctypes.data_as(_ip),
                       cz.ctypes.data_as(_ip), _ptr(w), _ptr(cs2))
    return cx, cy, cz, w, float(cs2[0])


def feq(rho, u, q=Q):
    out = np.zeros(q)
    _L().ora3q_feq(q, rho, _ptr(_f64(u, (3,))), _ptr(out))
    return out


def force_term(tau, rho, us, ustar, q=Q):
    out = np.zeros(q)
    _L().ora3q_force_term(q, tau, rho, _ptr(_f64(us, (3,))), _ptr(_f64(ustar, (3,))), _ptr(out))
    return out


def guo_term(tau, u, G, q=Q):
    out = np.zeros(q)
    _L().ora3q_guo_term(q, tau, _ptr(_f64(u, (3,))), _ptr(_f64(G, (3,))), _ptr(out))
    return out


def collide_node(tau, rho0, f_dev, phis=(), us=(), G=(0.0, 0.0, 0.0), force_mode=0, q=Q):
    """One node, no streaming.  Returns (status, fpost_dev, rho, u, ustar, force_b[nb, 3])."""
    nb = len(phis)
    ph = _f64(np.asarray(phis, np.float64).reshape(-1))
    usa = _f64(np.asarray(us, np.float64).reshape(nb, 3)) if nb else None
    fp = np.zeros(q)
    rho = np.zeros(1)
    u = np.zeros(3)
    ust = np.zeros(3)
    fb = np.zeros(max(nb, 1) * 3)
    st = _L().ora3q_collide_node(q, tau, rho0, _ptr(_f64(f_dev, (q,))), nb,
                                 _ptr(ph) if nb else None, _ptr(usa) if nb else None,
                                 _ptr(_f64(G, (3,))), force_mode, _ptr(fp), _ptr(rho), _ptr(u),
                                 _ptr(ust), _ptr(fb))
    return int(st), fp, float(rho[0]), u, ust, fb[: 3 * nb].reshape(nb, 3)


def nee_node(tau, rho0, f_nb_dev, G=(0.0, 0.0, 0.0), rho_set=None, u_set=None, q=Q):
    """Non-equilibrium extrapolation at one boundary node from its neighbour's populations:
    rho_set / u_set prescribe the boundary state, None takes the neighbour's.
    Returns (fpost_dev, rho_b, u_b)."""
    fp = np.zeros(q)
    rb = np.zeros(1)
    ub = np.zeros(3)
    us = _f64(u_set if u_set is not None else (0.0, 0.0, 0.0), (3,))
    _L().ora3q_nee_node(q, tau, rho0, _ptr(_f64(f_nb_dev, (q,))), _ptr(_f64(G, (3,))),
                        int(rho_set is None), float(rho_set or 0.0), int(u_set is None),
                        _ptr(us), _ptr(fp), _ptr(rb), _ptr(ub))
    return fp, float(rb[0]), ub


def inlet_shape(params, j, k):
    """The inlet profile factor of the inlet node (j, k)."""
    cp = params._c()
    return float(_L().ora3_inlet_shape(C.byref(cp), int(j), int(k)))


def pp_force(d, ri, rj, xi, eps_p, eps_p1):
    out = np.zeros(3)
    _L().ora3_pp_force(_ptr(_f64(d, (3,))), ri, rj, xi, eps_p, eps_p1, _ptr(out))
    return out


def pw_force(d, r, xi, eps_w, eps_w1):
    out = np.zeros(3)
    _L().ora3_pw_force(_ptr(_f64(d, (3,))), r, xi, eps_w, eps_w1, _ptr(out))
    return out


def body_update(m, I, F, T, x, u, om):
    x, u, om = (np.array(v, np.float64).reshape(3) for v in (x, u, om))
    _L().ora3_body_update(m, I, _ptr(_f64(F, (3,))), _ptr(_f64(T, (3,))), _ptr(x), _ptr(u),
                          _ptr(om))
    return x, u, om


@dataclass
class Oracle3Params:
    nx: int
    ny: int
    nz: int
    tau: float
    rho0: float = 1.0
    eps: float = 2.0
    cutoff: float = 4.0
    G: tuple = (0.0, 0.0, 0.0)
    g: tuple = (0.0, 0.0, 0.0)
    wall_mask: int = 0         # bit 0: y seam, bit 1: x seam, bit 2: z seam
    wall_h: float = 4.0
    force_mode: int = 0
    eps_p: float = 1.0e4
    eps_p1: float = 1.0e4
    eps_w: float = 0.5e4
    eps_w1: float = 0.5e4
    xi: float = 1.0
    lattice: int = 19          # 19: D3Q19, 27: D3Q27
    x_boundary: int = 0        # 1: inlet column x = 0, outlet column x = nx - 1
    inlet_kind: int = 0        # 0: velocity u_in; 1: density rho_in
    inlet_profile: int = 0     # 0 uniform; 1 parabolic across y; 2 across y and z
    outlet_kind: int = 0       # 0: density rho_out; 1: zero gradient
    u_in: tuple = (0.0, 0.0, 0.0)
    rho_in: float = 1.0
    rho_out: float = 1.0

    def _c(self):
        p = _Params()
        p.nx, p.ny, p.nz = int(self.nx), int(self.ny), int(self.nz)
        p.tau, p.rho0, p.eps, p.cutoff = self.tau, self.rho0, self.eps, self.cutoff
        for a in range(3):
            p.G[a] = self.G[a]
            p.g[a] = self.g[a]
        p.wall_mask = int(self.wall_mask)
        p.wall_h = self.wall_h
        p.force_mode = int(self.force_mode)
        p.eps_p, p.eps_p1, p.eps_w, p.eps_w1, p.xi = (self.eps_p, self.eps_p1, self.eps_w,
                                                      self.eps_w1, self.xi)
        p.lattice = int(self.lattice)
        p.x_boundary, p.inlet_kind = int(self.x_boundary), int(self.inlet_kind)
        p.inlet_profile, p.outlet_kind = int(self.inlet_profile), int(self.outlet_kind)
        for a in range(3):
            p.u_in[a] = self.u_in[a]
        p.rho_in, p.rho_out = self.rho_in, self.rho_out
        return p


class Oracle3Error(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


class Oracle3Solver:
    """FP64 3-D DI-LBM solver.  Populations: deviations, shape [q, nz, ny, nx], q = 19 or
    27 (params.lattice)."""

    def __init__(self, params: Oracle3Params):
        self.params = params
        h = C.c_void_p()
        cp = params._c()
        st = _L().ora3_create(C.byref(cp), C.byref(h))
        if st != 0:
            raise Oracle3Error(st, "ora3_create")
        self._h = h
        self.nb = 0

    def close(self):
        if getattr(self, "_h", None):
            _L().ora3_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what):
        if st != 0:
            raise Oracle3Error(st, what)

    @property
    def shape(self):
        p = self.params
        return (p.nz, p.ny, p.nx)

    def set_particles(self, pos, radius, density, vel=None, omega=None, fixed=None):
        pos = _f64(pos, (-1, 3))
        n = pos.shape[0]
        radius = _f64(radius, (n,))
        density = _f64(density, (n,))
        vel = _f64(vel, (n, 3)) if vel is not None else None
        omega = _f64(omega, (n, 3)) if omega is not None else None
        fx = (np.ascontiguousarray(fixed, dtype=np.uint8).reshape(n)
              if fixed is not None else None)
        st = _L().ora3_set_particles(self._h, n, _ptr(pos), _ptr(vel), _ptr(omega),
                                     _ptr(radius), _ptr(density),
                                     fx.ctypes.data_as(_u8p) if fx is not None else None)
        self._check(st, "ora3_set_particles")
        self.nb = n

    def set_populations(self, f_dev):
        f_dev = _f64(f_dev, (self.params.lattice,) + self.shape)
        self._check(_L().ora3_set_populations(self._h, _ptr(f_dev)), "ora3_set_populations")

    def get_populations(self):
        out = np.zeros((self.params.lattice,) + self.shape)
        self._check(_L().ora3_get_populations(self._h, _ptr(out)), "ora3_get_populations")
        return out

    def step(self, n=1):
        self._check(_L().ora3_step(self._h, int(n)), "ora3_step")

    def step_status(self, n=1):
        return int(_L().ora3_step(self._h, int(n)))

    def get_fields(self):
        rho, ux, uy, uz = (np.zeros(self.shape) for _ in range(4))
        self._check(_L().ora3_get_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz)),
                    "ora3_get_fields")
        return rho, ux, uy, uz

    def get_particle_forces(self):
        f = np.zeros((max(self.nb, 1), 3))
        t = np.zeros((max(self.nb, 1), 3))
        self._check(_L().ora3_get_particle_forces(self._h, _ptr(f), _ptr(t)),
                    "ora3_get_particle_forces")
        return f[: self.nb], t[: self.nb]

    def get_particles(self):
        x, u, w = (np.zeros((max(self.nb, 1), 3)) for _ in range(3))
        self._check(_L().ora3_get_particles(self._h, _ptr(x), _ptr(u), _ptr(w)),
                    "ora3_get_particles")
        return x[: self.nb], u[: self.nb], w[: self.nb]

    def get_wall_force(self):
        f = np.zeros(3)
        self._check(_L().ora3_get_wall_force(self._h, _ptr(f)), "ora3_get_wall_force")
        return f
