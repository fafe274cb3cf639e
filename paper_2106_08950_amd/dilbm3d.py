"""Thin ctypes binding of the three-dimensional DI-LBM calls of libdilbm.so (the C ABI
declared in include/dilbm3d.h: D3Q19 or D3Q27 lattice, spherical particles, FP32 or FP16
population storage, optional open ends in x).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
Loading fails loudly when the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import dilbm

Q = 19
ABI_VERSION = 4
WALL_Y, WALL_X, WALL_Z = 1, 2, 4

EXPORTED = [
    "dilbm3d_params_init", "dilbm3d_create", "dilbm3d_set_particles",
    "dilbm3d_set_populations", "dilbm3d_get_populations", "dilbm3d_step",
    "dilbm3d_get_fields", "dilbm3d_get_particle_forces", "dilbm3d_get_particles",
    "dilbm3d_get_wall_force", "dilbm3d_get_step_count", "dilbm3d_set_kernel_timing",
    "dilbm3d_get_kernel_timing", "dilbm3d_get_kernel_launch_times", "dilbm3d_destroy", "dilbm3d_last_error",
    "dilbm3d_batch_create", "dilbm3d_batch_step", "dilbm3d_batch_destroy", "dilbm3d_batch_last_error",
]


class dilbm3d_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("interface_width", C.c_double), ("phi_cutoff", C.c_double),
        ("body_force", C.c_double * 3), ("gravity", C.c_double * 3),
        ("wall_mask", C.c_uint32), ("wall_half_thickness", C.c_double),
        ("force_mode", C.c_int32),
        ("coll_eps_p", C.c_double), ("coll_eps_p_overlap", C.c_double),
        ("coll_eps_w", C.c_double), ("coll_eps_w_overlap", C.c_double),
        ("coll_xi", C.c_double),
        ("list_capacity", C.c_int32), ("lattice", C.c_int32), ("storage", C.c_int32),
        ("fp16_scale_log2", C.c_int32),
        ("x_boundary", C.c_int32), ("inlet_kind", C.c_int32), ("inlet_profile", C.c_int32),
        ("outlet_kind", C.c_int32), ("inlet_velocity", C.c_double * 3),
        ("inlet_density", C.c_double), ("outlet_density", C.c_double),
        ("device", C.c_int32), ("stream", C.c_void_p),
    ]


_dp = C.POINTER(C.c_double)
_bound = None


def load():
    """Bind the dilbm3d_* entry points of libdilbm.so (raises if it has not been built)."""
    global _bound
    if _bound is not None:
        return _bound
    lib = dilbm.load()
    V, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER(dilbm3d_params)
    sig = {
        "dilbm3d_params_init": (I32, [P]),
        "dilbm3d_create": (I32, [P, C.POINTER(V)]),
        "dilbm3d_set_particles": (I32, [V, I32, _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_uint8)]),
        "dilbm3d_set_populations": (I32, [V, _dp]),
        "dilbm3d_get_populations": (I32, [V, _dp]),
        "dilbm3d_step": (I32, [V, I64]),
        "dilbm3d_get_fields": (I32, [V, _dp, _dp, _dp, _dp]),
        "dilbm3d_get_particle_forces": (I32, [V, _dp, _dp]),
        "dilbm3d_get_particles": (I32, [V, _dp, _dp, _dp]),
        "dilbm3d_get_wall_force": (I32, [V, _dp]),
        "dilbm3d_get_step_count": (I32, [V, C.POINTER(I64)]),
        "dilbm3d_set_kernel_timing": (I32, [V, I32]),
        "dilbm3d_get_kernel_timing": (I32, [V, C.POINTER(D), C.POINTER(I64)]),
        "dilbm3d_get_kernel_launch_times": (I32, [V, _dp, I64, C.POINTER(I64)]),
        "dilbm3d_destroy": (None, [V]),
        "dilbm3d_last_error": (C.c_char_p, [V]),
        "dilbm3d_batch_create": (I32, [C.POINTER(V), I32, C.POINTER(V)]),
        "dilbm3d_batch_step": (I32, [V, I64]),
        "dilbm3d_batch_destroy": (None, [V]),
        "dilbm3d_batch_last_error": (C.c_char_p, [V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _bound = lib
    return lib


@dataclass
class Params3D:
    nx: int
    ny: int
    nz: int
    tau: float
    rho0: float = 1.0
    interface_width: float = 2.0
    phi_cutoff: float = 4.0
    body_force: tuple = (0.0, 0.0, 0.0)
    gravity: tuple = (0.0, 0.0, 0.0)
    wall_mask: int = 0
    wall_half_thickness: float = 4.0
    force_mode: int = dilbm.FORCE_MOMENTUM_EXCHANGE
    coll_eps_p: float = 1.0e4
    coll_eps_p_overlap: float = 1.0e4
    coll_eps_w: float = 0.5e4
    coll_eps_w_overlap: float = 0.5e4
    coll_xi: float = 1.0
    list_capacity: int = 0
    lattice: int = 19          # 19: D3Q19, 27: D3Q27
    storage: int = 0           # 0: FP32 populations, 1: FP16 (dilbm.STORE_FP16)
    fp16_scale_log2: int = dilbm.FP16_SCALE_AUTO  # or k in [0, 24]
    x_boundary: int = 0        # dilbm.XBC_*: 1 = inlet plane x = 0, outlet plane x = nx - 1
    inlet_kind: int = 0        # dilbm.INLET_VELOCITY or dilbm.INLET_PRESSURE
    inlet_profile: int = 0     # 0 uniform; 1 parabolic across y; 2 across y and z
    outlet_kind: int = 0       # dilbm.OUTLET_PRESSURE or dilbm.OUTLET_ZERO_GRADIENT
    inlet_velocity: tuple = (0.0, 0.0, 0.0)
    inlet_density: float = 1.0
    outlet_density: float = 1.0
    device: int = 0
    stream: int = 0
    abi_version: int = ABI_VERSION

    def to_c(self) -> dilbm3d_params:
        p = dilbm3d_params()
        load().dilbm3d_params_init(C.byref(p))
        p.abi_version = int(self.abi_version)
        p.nx, p.ny, p.nz = int(self.nx), int(self.ny), int(self.nz)
        p.tau, p.rho0 = float(self.tau), float(self.rho0)
        p.interface_width, p.phi_cutoff = float(self.interface_width), float(self.phi_cutoff)
        for a in range(3):
            p.body_force[a] = float(self.body_force[a])
            p.gravity[a] = float(self.gravity[a])
        p.wall_mask = int(self.wall_mask)
        p.wall_half_thickness = float(self.wall_half_thickness)
        p.force_mode = int(self.force_mode)
        p.coll_eps_p, p.coll_eps_p_overlap = float(self.coll_eps_p), float(self.coll_eps_p_overlap)
        p.coll_eps_w, p.coll_eps_w_overlap = float(self.coll_eps_w), float(self.coll_eps_w_overlap)
        p.coll_xi = float(self.coll_xi)
        p.list_capacity = int(self.list_capacity)
        p.lattice = int(self.lattice)
        p.storage = int(self.storage)
        p.fp16_scale_log2 = int(self.fp16_scale_log2)
        p.x_boundary, p.inlet_kind = int(self.x_boundary), int(self.inlet_kind)
        p.inlet_profile, p.outlet_kind = int(self.inlet_profile), int(self.outlet_kind)
        for a in range(3):
            p.inlet_velocity[a] = float(self.inlet_velocity[a])
        p.inlet_density, p.outlet_density = float(self.inlet_density), float(self.outlet_density)
        p.device = int(self.device)
        p.stream = int(self.stream) or None
        return p


def params_from_workload(wl, **kw) -> Params3D:
    """Params3D of an inputs3d.Workload3D; keyword arguments override fields."""
    p = Params3D(nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, rho0=wl.rho0,
                 interface_width=wl.eps, phi_cutoff=wl.cutoff, body_force=tuple(wl.G),
                 gravity=tuple(wl.g), wall_mask=wl.wall_mask, wall_half_thickness=wl.wall_h,
                 force_mode=wl.force_mode, coll_eps_p=wl.eps_p, coll_eps_p_overlap=wl.eps_p1,
                 coll_eps_w=wl.eps_w, coll_eps_w_overlap=wl.eps_w1, coll_xi=wl.xi,
                 x_boundary=wl.x_boundary, inlet_kind=wl.inlet_kind,
                 inlet_profile=wl.inlet_profile, outlet_kind=wl.outlet_kind,
                 inlet_velocity=tuple(wl.u_in), inlet_density=wl.rho_in,
                 outlet_density=wl.rho_out)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


class Solver3D:
    """One 3-D DI-LBM solve on the GPU.  Populations: [q, nz, ny, nx] deviations, q = 19
    (D3Q19) or 27 (D3Q27, params.lattice = 27)."""

    def __init__(self, params: Params3D):
        self.params = params
        lib = load()
        h = C.c_void_p()
        cp = params.to_c()
        st = lib.dilbm3d_create(C.byref(cp), C.byref(h))
        if st != 0:
            raise dilbm.DilbmError(st, "dilbm3d_create", lib.dilbm3d_last_error(None).decode())
        self._h = h
        self.nb = 0

    @property
    def shape(self):
        p = self.params
        return (p.nz, p.ny, p.nx)

    @property
    def q(self):
        return 27 if self.params.lattice == 27 else 19

    def _check(self, st, where):
        if st != 0:
            raise dilbm.DilbmError(st, where, load().dilbm3d_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().dilbm3d_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_particles(self, pos, radius, density, vel=None, omega=None, fixed=None):
        pos = _f64(pos, (-1, 3))
        n = pos.shape[0]
        radius = _f64(radius, (n,))
        density = _f64(density, (n,))
        vel = _f64(vel, (n, 3)) if vel is not None else None
        omega = _f64(omega, (n, 3)) if omega is not None else None
        fx = np.ascontiguousarray(fixed, dtype=np.uint8).reshape(n) if fixed is not None else None
        self._check(load().dilbm3d_set_particles(
            self._h, n, _ptr(pos), _ptr(vel), _ptr(omega), _ptr(radius), _ptr(density),
            fx.ctypes.data_as(C.POINTER(C.c_uint8)) if fx is not None else None),
            "dilbm3d_set_particles")
        self.nb = n

    def set_populations(self, f_dev):
        f_dev = _f64(f_dev, (self.q,) + self.shape)
        self._check(load().dilbm3d_set_populations(self._h, _ptr(f_dev)), "dilbm3d_set_populations")

    def get_populations(self):
        out = np.zeros((self.q,) + self.shape)
        self._check(load().dilbm3d_get_populations(self._h, _ptr(out)), "dilbm3d_get_populations")
        return out

    def step(self, n=1):
        self._check(load().dilbm3d_step(self._h, int(n)), "dilbm3d_step")

    def step_status(self, n=1) -> int:
        return int(load().dilbm3d_step(self._h, int(n)))

    def get_fields(self):
        rho, ux, uy, uz = (np.zeros(self.shape) for _ in range(4))
        self._check(load().dilbm3d_get_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz)),
                    "dilbm3d_get_fields")
        return rho, ux, uy, uz

    def get_particle_forces(self):
        f = np.zeros((max(self.nb, 1), 3))
        t = np.zeros((max(self.nb, 1), 3))
        self._check(load().dilbm3d_get_particle_forces(self._h, _ptr(f), _ptr(t)),
                    "dilbm3d_get_particle_forces")
        return f[: self.nb], t[: self.nb]

    def get_particles(self):
        x, u, w = (np.zeros((max(self.nb, 1), 3)) for _ in range(3))
        self._check(load().dilbm3d_get_particles(self._h, _ptr(x), _ptr(u), _ptr(w)),
                    "dilbm3d_get_particles")
        return x[: self.nb], u[: self.nb], w[: self.nb]

    def step_count(self) -> int:
        v = C.c_int64(0)
        self._check(load().dilbm3d_get_step_count(self._h, C.byref(v)), "dilbm3d_get_step_count")
        return v.value

    def get_wall_force(self):
        f = np.zeros(3)
        self._check(load().dilbm3d_get_wall_force(self._h, _ptr(f)), "dilbm3d_get_wall_force")
        return f

    def set_kernel_timing(self, on: bool):
        self._check(load().dilbm3d_set_kernel_timing(self._h, int(bool(on))),
                    "dilbm3d_set_kernel_timing")

    def kernel_timing(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(load().dilbm3d_get_kernel_timing(self._h, C.byref(ms), C.byref(n)),
                    "dilbm3d_get_kernel_timing")
        return ms.value, n.value

    def kernel_launch_times(self):
        """Every timed collide launch since timing was enabled (milliseconds)."""
        n = C.c_int64()
        self._check(load().dilbm3d_get_kernel_launch_times(self._h, None, 0, C.byref(n)),
                    "dilbm3d_get_kernel_launch_times")
        out = np.zeros(max(int(n.value), 1))
        self._check(load().dilbm3d_get_kernel_launch_times(self._h, _ptr(out), int(n.value),
                                                           C.byref(n)),
                    "dilbm3d_get_kernel_launch_times")
        return out[: int(n.value)]


class Batch3D:
    """Several Solver3D advanced together (dilbm3d_batch_*): one collide launch and one
    sphere launch per step over all members.  The batch keeps references to its members;
    once a member is closed the batch refuses to step (it may still be closed)."""

    def __init__(self, members):
        self.members = list(members)
        lib = load()
        arr = (C.c_void_p * len(self.members))(*[m._h.value if m._h else None
                                                 for m in self.members])
        h = C.c_void_p()
        st = lib.dilbm3d_batch_create(arr, len(self.members), C.byref(h))
        if st != 0:
            raise dilbm.DilbmError(st, "dilbm3d_batch_create",
                                   lib.dilbm3d_batch_last_error(None).decode())
        self._h = h

    def step(self, n=1):
        if not self._h:
            raise dilbm.DilbmError(dilbm.ESTATE, "dilbm3d_batch_step", "the batch is closed")
        if not all(m._h for m in self.members):
            # the library would step through a destroyed member; refuse here instead
            raise dilbm.DilbmError(dilbm.ESTATE, "dilbm3d_batch_step",
                                   "a member was closed while the batch is open")
        st = load().dilbm3d_batch_step(self._h, int(n))
        if st != 0:
            raise dilbm.DilbmError(st, "dilbm3d_batch_step",
                                   load().dilbm3d_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().dilbm3d_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
