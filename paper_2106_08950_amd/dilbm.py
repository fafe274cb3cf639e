"""Thin ctypes binding of libdilbm.so (the C ABI declared in include/dilbm.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
The library must have been built (``python -m paper_2106_08950_amd.build``); loading
fails loudly when it is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdilbm.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE, EABI, ECAPACITY, EAGAIN = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSTABLE",
                -5: "ESTATE", -6: "EABI", -7: "ECAPACITY", -8: "EAGAIN"}
STORE_FP32, STORE_FP16 = 0, 1
FP16_SCALE_AUTO = -1  # fp16_scale_log2: the library picks the scale (DILBM_FP16_SCALE_AUTO)
FORCE_MOMENTUM_EXCHANGE, FORCE_PAPER_LITERAL = 0, 1
WALL_Y, WALL_X = 1, 2
XBC_PERIODIC, XBC_INLET_OUTLET = 0, 1
INLET_VELOCITY, INLET_PRESSURE = 0, 1
OUTLET_PRESSURE, OUTLET_ZERO_GRADIENT = 0, 1
ABI_VERSION = 2

EXPORTED = [
    "dilbm_params_init", "dilbm_num_tile_shapes", "dilbm_tile_shape", "dilbm_footprint",
    "dilbm_create", "dilbm_set_particles", "dilbm_set_populations", "dilbm_get_populations",
    "dilbm_step", "dilbm_get_fields", "dilbm_get_fields_region",
    "dilbm_get_fields_region_noalloc", "dilbm_get_particle_forces",
    "dilbm_get_particles",
    "dilbm_get_wall_force", "dilbm_get_step_count", "dilbm_get_body_count",
    "dilbm_set_kernel_timing",
    "dilbm_get_kernel_timing", "dilbm_get_kernel_launch_times", "dilbm_destroy",
    "dilbm_last_error",
    "dilbm_pool_create", "dilbm_pool_submit", "dilbm_pool_run", "dilbm_pool_sync",
    "dilbm_pool_query", "dilbm_pool_get_fields", "dilbm_pool_get_particles",
    "dilbm_pool_get_particle_forces", "dilbm_pool_release", "dilbm_pool_set_launch",
    "dilbm_pool_autotune", "dilbm_pool_stats", "dilbm_pool_last_error", "dilbm_pool_destroy",
]


class dilbm_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("interface_width", C.c_double), ("phi_cutoff", C.c_double),
        ("body_force", C.c_double * 2), ("gravity", C.c_double * 2),
        ("wall_mask", C.c_uint32), ("wall_half_thickness", C.c_double),
        ("force_mode", C.c_int32),
        ("coll_eps_p", C.c_double), ("coll_eps_p_overlap", C.c_double),
        ("coll_eps_w", C.c_double), ("coll_eps_w_overlap", C.c_double),
        ("coll_xi", C.c_double),
        ("storage", C.c_int32), ("fp16_scale_log2", C.c_int32),
        ("list_capacity", C.c_int32), ("tile", C.c_int32),
        ("x_boundary", C.c_int32), ("inlet_kind", C.c_int32), ("inlet_profile", C.c_int32),
        ("outlet_kind", C.c_int32), ("inlet_velocity", C.c_double * 2),
        ("inlet_density", C.c_double), ("outlet_density", C.c_double),
        ("device", C.c_int32), ("stream", C.c_void_p),
    ]


class DilbmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str = ""):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} {message}".strip())
        self.status = status


_dp = C.POINTER(C.c_double)
_lib = None


def load():
    """Load libdilbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libdilbm.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_2106_08950_amd.build` (no fallback exists)")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch first makes
    # the library bind to that one runtime, so torch streams and device pointers are valid
    # handles here; loaded the other way round a process would hold two runtimes and
    # torch would find no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    V, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    P = C.POINTER(dilbm_params)
    sig = {
        "dilbm_params_init": (None, [P]),
        "dilbm_num_tile_shapes": (I32, []),
        "dilbm_tile_shape": (I32, [I32, C.POINTER(I32), C.POINTER(I32)]),
        "dilbm_footprint": (I32, [P, I32, C.POINTER(U64)]),
        "dilbm_create": (I32, [P, C.POINTER(V)]),
        "dilbm_set_particles": (I32, [V, I32, _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_uint8)]),
        "dilbm_set_populations": (I32, [V, _dp]),
        "dilbm_get_populations": (I32, [V, _dp]),
        "dilbm_step": (I32, [V, I64]),
        "dilbm_get_fields": (I32, [V, _dp, _dp, _dp]),
        "dilbm_get_fields_region": (I32, [V, I32, I32, I32, I32, _dp, _dp, _dp]),
        "dilbm_get_fields_region_noalloc": (I32, [V, I32, I32, I32, I32, _dp, _dp, _dp]),
        "dilbm_get_particle_forces": (I32, [V, _dp, _dp]),
        "dilbm_get_particles": (I32, [V, _dp, _dp, _dp]),
        "dilbm_get_wall_force": (I32, [V, _dp]),
        "dilbm_get_step_count": (I32, [V, C.POINTER(I64)]),
        "dilbm_get_body_count": (I32, [V, C.POINTER(I32)]),
        "dilbm_set_kernel_timing": (I32, [V, I32]),
        "dilbm_get_kernel_timing": (I32, [V, C.POINTER(D), C.POINTER(I64)]),
        "dilbm_get_kernel_launch_times": (I32, [V, _dp, I64, C.POINTER(I64)]),
        "dilbm_destroy": (None, [V]),
        "dilbm_last_error": (C.c_char_p, [V]),
        "dilbm_pool_create": (I32, [I32, V, V, U64, C.POINTER(V)]),
        "dilbm_pool_submit": (I32, [V, P, I32, _dp, _dp, _dp, _dp, _dp,
                                    C.POINTER(C.c_uint8), I64, C.POINTER(I64)]),
        "dilbm_pool_run": (I32, [V, I32]),
        "dilbm_pool_sync": (I32, [V]),
        "dilbm_pool_query": (I32, [V, I64, C.POINTER(I64), C.POINTER(I32)]),
        "dilbm_pool_get_fields": (I32, [V, I64, _dp, _dp, _dp]),
        "dilbm_pool_get_particles": (I32, [V, I64, _dp, _dp, _dp]),
        "dilbm_pool_get_particle_forces": (I32, [V, I64, _dp, _dp]),
        "dilbm_pool_release": (I32, [V, I64]),
        "dilbm_pool_set_launch": (I32, [V, I32, I32]),
        "dilbm_pool_autotune": (I32, [V, I32, C.POINTER(I32), C.POINTER(I32)]),
        "dilbm_pool_stats": (I32, [V, C.POINTER(U64), C.POINTER(I32)]),
        "dilbm_pool_last_error": (C.c_char_p, [V]),
        "dilbm_pool_destroy": (None, [V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


@dataclass
class Params:
    nx: int
    ny: int
    tau: float = 0.8
    rho0: float = 1.0
    interface_width: float = 2.0
    phi_cutoff: float = 4.0
    body_force: tuple = (0.0, 0.0)
    gravity: tuple = (0.0, 0.0)
    wall_mask: int = 0
    wall_half_thickness: float = 4.0
    force_mode: int = FORCE_MOMENTUM_EXCHANGE
    coll_eps_p: float = 1.0e4
    coll_eps_p_overlap: float = 1.0e4
    coll_eps_w: float = 0.5e4
    coll_eps_w_overlap: float = 0.5e4
    coll_xi: float = 1.0
    storage: int = STORE_FP32
    fp16_scale_log2: int = FP16_SCALE_AUTO  # or k in [0, 24]
    list_capacity: int = 0
    tile: int = -1
    x_boundary: int = XBC_PERIODIC
    inlet_kind: int = INLET_VELOCITY
    inlet_profile: int = 0
    outlet_kind: int = OUTLET_PRESSURE
    inlet_velocity: tuple = (0.0, 0.0)
    inlet_density: float = 1.0
    outlet_density: float = 1.0
    device: int = 0
    stream: int = 0

    def to_c(self) -> dilbm_params:
        p = dilbm_params()
        load().dilbm_params_init(C.byref(p))
        for name, _t in dilbm_params._fields_:
            if name == "abi_version":
                continue
            v = getattr(self, name)
            if name in ("body_force", "gravity", "inlet_velocity"):
                getattr(p, name)[0], getattr(p, name)[1] = float(v[0]), float(v[1])
            elif name == "stream":
                p.stream = C.c_void_p(int(v)) if v else None
            else:
                setattr(p, name, v)
        return p


def params_from_workload(wl, **overrides) -> Params:
    """Map an ``inputs.Workload`` onto the ABI parameters."""
    d = dict(nx=wl.nx, ny=wl.ny, tau=wl.tau, rho0=wl.rho0, interface_width=wl.eps,
             phi_cutoff=wl.cutoff, body_force=tuple(wl.G), gravity=tuple(wl.g),
             wall_mask=wl.wall_mask, wall_half_thickness=wl.wall_h, force_mode=wl.force_mode,
             coll_eps_p=wl.eps_p, coll_eps_p_overlap=wl.eps_p1, coll_eps_w=wl.eps_w,
             coll_eps_w_overlap=wl.eps_w1, coll_xi=wl.xi, x_boundary=wl.x_boundary,
             inlet_kind=wl.inlet_kind, inlet_profile=wl.inlet_profile,
             outlet_kind=wl.outlet_kind, inlet_velocity=tuple(wl.u_in),
             inlet_density=wl.rho_in, outlet_density=wl.rho_out)
    d.update(overrides)
    return Params(**d)


def tile_shapes():
    lib = load()
    out = []
    for i in range(lib.dilbm_num_tile_shapes()):
        tx, ty = C.c_int32(), C.c_int32()
        lib.dilbm_tile_shape(i, C.byref(tx), C.byref(ty))
        out.append((tx.value, ty.value))
    return out


def footprint(params: Params, n_bodies: int) -> int:
    b = C.c_uint64()
    cp = params.to_c()
    st = load().dilbm_footprint(C.byref(cp), int(n_bodies), C.byref(b))
    if st != OK:
        raise DilbmError(st, "dilbm_footprint")
    return int(b.value)


class Solver:
    """One DI-LBM solve on the GPU (dilbm_create ... dilbm_destroy)."""

    def __init__(self, params: Params):
        self.params = params
        self._lib = load()
        h = C.c_void_p()
        cp = params.to_c()
        st = self._lib.dilbm_create(C.byref(cp), C.byref(h))
        if st != OK:
            raise DilbmError(st, "dilbm_create", self._lib.dilbm_last_error(None).decode())
        self._h = h
        self.nb = 0

    def _check(self, st, where):
        if st != OK:
            raise DilbmError(st, where, self._lib.dilbm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dilbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_particles(self, pos, radius, density, vel=None, omega=None, fixed=None):
        pos = _f64(pos, (-1, 2))
        n = pos.shape[0]
        fx = np.ascontiguousarray(fixed, np.uint8).reshape(n) if fixed is not None else None
        st = self._lib.dilbm_set_particles(
            self._h, n, _ptr(pos), _ptr(_f64(vel, (n, 2)) if vel is not None else None),
            _ptr(_f64(omega, (n,)) if omega is not None else None), _ptr(_f64(radius, (n,))),
            _ptr(_f64(density, (n,))),
            fx.ctypes.data_as(C.POINTER(C.c_uint8)) if fx is not None else None)
        self.nb = self.body_count()  # the library's count, whatever the status
        self._check(st, "dilbm_set_particles")

    def body_count(self) -> int:
        v = C.c_int32()
        self._check(self._lib.dilbm_get_body_count(self._h, C.byref(v)), "dilbm_get_body_count")
        return int(v.value)

    def set_populations(self, f_dev):
        p = self.params
        f_dev = _f64(f_dev, (9, p.ny, p.nx))
        self._check(self._lib.dilbm_set_populations(self._h, _ptr(f_dev)),
                    "dilbm_set_populations")

    def get_populations(self):
        p = self.params
        out = np.empty((9, p.ny, p.nx))
        self._check(self._lib.dilbm_get_populations(self._h, _ptr(out)), "dilbm_get_populations")
        return out

    def step(self, n=1):
        self._check(self._lib.dilbm_step(self._h, int(n)), "dilbm_step")

    def step_status(self, n=1) -> int:
        return int(self._lib.dilbm_step(self._h, int(n)))

    def get_fields(self):
        p = self.params
        rho = np.empty((p.ny, p.nx))
        ux = np.empty((p.ny, p.nx))
        uy = np.empty((p.ny, p.nx))
        self._check(self._lib.dilbm_get_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy)),
                    "dilbm_get_fields")
        return rho, ux, uy

    def get_fields_region(self, x0, y0, w, h):
        rho = np.empty((h, w))
        ux = np.empty((h, w))
        uy = np.empty((h, w))
        self._check(self._lib.dilbm_get_fields_region(self._h, int(x0), int(y0), int(w), int(h),
                                                      _ptr(rho), _ptr(ux), _ptr(uy)),
                    "dilbm_get_fields_region")
        return rho, ux, uy

    def get_fields_region_noalloc(self, x0, y0, w, h):
        """dilbm_get_fields_region_noalloc: the same values through the library's fixed
        staging array (no device allocation)."""
        rho = np.empty((h, w))
        ux = np.empty((h, w))
        uy = np.empty((h, w))
        self._check(self._lib.dilbm_get_fields_region_noalloc(
            self._h, int(x0), int(y0), int(w), int(h), _ptr(rho), _ptr(ux), _ptr(uy)),
            "dilbm_get_fields_region_noalloc")
        return rho, ux, uy

    def get_particle_forces(self):
        f = np.zeros((max(self.nb, 1), 2))
        t = np.zeros(max(self.nb, 1))
        self._check(self._lib.dilbm_get_particle_forces(self._h, _ptr(f), _ptr(t)),
                    "dilbm_get_particle_forces")
        return f[: self.nb], t[: self.nb]

    def get_particles(self):
        x = np.zeros((max(self.nb, 1), 2))
        u = np.zeros((max(self.nb, 1), 2))
        w = np.zeros(max(self.nb, 1))
        self._check(self._lib.dilbm_get_particles(self._h, _ptr(x), _ptr(u), _ptr(w)),
                    "dilbm_get_particles")
        return x[: self.nb], u[: self.nb], w[: self.nb]

    def get_wall_force(self):
        f = np.zeros(2)
        self._check(self._lib.dilbm_get_wall_force(self._h, _ptr(f)), "dilbm_get_wall_force")
        return f

    def step_count(self) -> int:
        v = C.c_int64()
        self._check(self._lib.dilbm_get_step_count(self._h, C.byref(v)), "dilbm_get_step_count")
        return int(v.value)

    def set_kernel_timing(self, on: bool):
        self._check(self._lib.dilbm_set_kernel_timing(self._h, 1 if on else 0),
                    "dilbm_set_kernel_timing")

    def kernel_timing(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self._lib.dilbm_get_kernel_timing(self._h, C.byref(ms), C.byref(n)),
                    "dilbm_get_kernel_timing")
        return float(ms.value), int(n.value)

    def kernel_launch_times(self):
        """Every timed collide launch since timing was enabled (milliseconds)."""
        n = C.c_int64()
        self._check(self._lib.dilbm_get_kernel_launch_times(self._h, None, 0, C.byref(n)),
                    "dilbm_get_kernel_launch_times")
        out = np.zeros(max(int(n.value), 1))
        self._check(self._lib.dilbm_get_kernel_launch_times(self._h, _ptr(out), int(n.value),
                                                            C.byref(n)),
                    "dilbm_get_kernel_launch_times")
        return out[: int(n.value)]


class Pool:
    """Many solves advanced together (dilbm_pool_*)."""

    def __init__(self, arena_bytes: int, device: int = 0, stream: int = 0, arena_ptr: int = 0):
        self._lib = load()
        h = C.c_void_p()
        st = self._lib.dilbm_pool_create(int(device), C.c_void_p(stream) if stream else None,
                                         C.c_void_p(arena_ptr) if arena_ptr else None,
                                         int(arena_bytes), C.byref(h))
        if st != OK:
            raise DilbmError(st, "dilbm_pool_create", self._lib.dilbm_last_error(None).decode())
        self._h = h
        self._nb = {}
        self._shape = {}

    def _check(self, st, where):
        if st != OK:
            raise DilbmError(st, where, self._lib.dilbm_pool_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dilbm_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, params: Params, nsteps: int, pos=None, radius=None, density=None, vel=None,
               omega=None, fixed=None):
        """Returns a ticket, or None when the arena has no room now (EAGAIN)."""
        pos = _f64(pos if pos is not None else np.zeros((0, 2)), (-1, 2))
        n = pos.shape[0]
        radius = _f64(radius if radius is not None else np.zeros(0), (n,))
        density = _f64(density if density is not None else np.zeros(0), (n,))
        fx = np.ascontiguousarray(fixed, np.uint8).reshape(n) if fixed is not None else None
        cp = params.to_c()
        t = C.c_int64()
        st = self._lib.dilbm_pool_submit(
            self._h, C.byref(cp), n, _ptr(pos),
            _ptr(_f64(vel, (n, 2)) if vel is not None else None),
            _ptr(_f64(omega, (n,)) if omega is not None else None), _ptr(radius), _ptr(density),
            fx.ctypes.data_as(C.POINTER(C.c_uint8)) if fx is not None else None, int(nsteps),
            C.byref(t))
        if st == EAGAIN:
            return None
        self._check(st, "dilbm_pool_submit")
        self._nb[t.value] = n
        self._shape[t.value] = (params.ny, params.nx)
        return int(t.value)

    def run(self, steps: int):
        self._check(self._lib.dilbm_pool_run(self._h, int(steps)), "dilbm_pool_run")

    def sync(self):
        self._check(self._lib.dilbm_pool_sync(self._h), "dilbm_pool_sync")

    def query(self, ticket: int):
        s = C.c_int64()
        d = C.c_int32()
        self._check(self._lib.dilbm_pool_query(self._h, int(ticket), C.byref(s), C.byref(d)),
                    "dilbm_pool_query")
        return int(s.value), bool(d.value)

    def get_fields(self, ticket: int):
        ny, nx = self._shape[ticket]
        rho = np.empty((ny, nx))
        ux = np.empty((ny, nx))
        uy = np.empty((ny, nx))
        self._check(self._lib.dilbm_pool_get_fields(self._h, int(ticket), _ptr(rho), _ptr(ux),
                                                    _ptr(uy)), "dilbm_pool_get_fields")
        return rho, ux, uy

    def get_particles(self, ticket: int):
        n = self._nb[ticket]
        x = np.zeros((max(n, 1), 2))
        u = np.zeros((max(n, 1), 2))
        w = np.zeros(max(n, 1))
        self._check(self._lib.dilbm_pool_get_particles(self._h, int(ticket), _ptr(x), _ptr(u),
                                                       _ptr(w)), "dilbm_pool_get_particles")
        return x[:n], u[:n], w[:n]

    def get_particle_forces(self, ticket: int):
        n = self._nb[ticket]
        f = np.zeros((max(n, 1), 2))
        t = np.zeros(max(n, 1))
        self._check(self._lib.dilbm_pool_get_particle_forces(self._h, int(ticket), _ptr(f),
                                                             _ptr(t)),
                    "dilbm_pool_get_particle_forces")
        return f[:n], t[:n]

    def release(self, ticket: int):
        self._check(self._lib.dilbm_pool_release(self._h, int(ticket)), "dilbm_pool_release")
        self._nb.pop(ticket, None)
        self._shape.pop(ticket, None)

    def set_launch(self, graph_steps: int, tile: int = -1):
        self._check(self._lib.dilbm_pool_set_launch(self._h, int(graph_steps), int(tile)),
                    "dilbm_pool_set_launch")

    def autotune(self, steps_per_trial: int = 32):
        k = C.c_int32()
        t = C.c_int32()
        self._check(self._lib.dilbm_pool_autotune(self._h, int(steps_per_trial), C.byref(k),
                                                  C.byref(t)), "dilbm_pool_autotune")
        return int(k.value), int(t.value)

    def stats(self):
        fb = C.c_uint64()
        m = C.c_int32()
        self._check(self._lib.dilbm_pool_stats(self._h, C.byref(fb), C.byref(m)),
                    "dilbm_pool_stats")
        return int(fb.value), int(m.value)
