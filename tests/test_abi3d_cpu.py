"""The three-dimensional C ABI (include/dilbm3d.h) on the CPU: the library exports every
declared symbol and rejects bad arguments before touching a device (no compute calls)."""
import ctypes as C
import os
import re

import pytest

from paper_2106_08950_amd import dilbm, dilbm3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dilbm3d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dilbm3d_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_what_the_binding_knows():
    assert _declared() == sorted(dilbm3d.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = dilbm3d.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_params_defaults():
    lib = dilbm3d.load()
    p = dilbm3d.dilbm3d_params()
    assert lib.dilbm3d_params_init(C.byref(p)) == dilbm.OK
    assert p.abi_version == dilbm3d.ABI_VERSION
    assert (p.rho0, p.interface_width, p.phi_cutoff, p.wall_half_thickness) == (1.0, 2.0, 4.0, 4.0)
    assert (p.coll_eps_p, p.coll_eps_p_overlap, p.coll_eps_w, p.coll_eps_w_overlap, p.coll_xi) == (
        1.0e4, 1.0e4, 0.5e4, 0.5e4, 1.0)
    assert (p.list_capacity, p.device, p.wall_mask) == (0, 0, 0)
    assert (p.storage, p.fp16_scale_log2) == (dilbm.STORE_FP32, dilbm.FP16_SCALE_AUTO)
    assert (p.x_boundary, p.inlet_density, p.outlet_density) == (dilbm.XBC_PERIODIC, 1.0, 1.0)
    assert p.stream is None
    assert lib.dilbm3d_params_init(None) == dilbm.EINVAL


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(nz=0), dict(nx=400, ny=400, nz=400), dict(tau=0.5),
    dict(tau=float("nan")), dict(rho0=0.0), dict(interface_width=0.0), dict(phi_cutoff=-1.0),
    dict(wall_mask=8), dict(wall_mask=4, wall_half_thickness=0.0), dict(force_mode=2),
    dict(list_capacity=5000), dict(coll_xi=-1.0), dict(coll_eps_p=0.0), dict(storage=2),
    dict(fp16_scale_log2=30), dict(fp16_scale_log2=-2),
    dict(body_force=(0.0, float("inf"), 0.0)), dict(gravity=(0.0, 0.0, float("nan"))),
    # open ends in x
    dict(x_boundary=2), dict(x_boundary=1, nx=2), dict(x_boundary=1, wall_mask=2),
    dict(x_boundary=1, inlet_kind=2), dict(x_boundary=1, outlet_kind=2),
    dict(x_boundary=1, inlet_profile=3), dict(x_boundary=1, inlet_profile=-1),
    dict(x_boundary=1, inlet_velocity=(float("nan"), 0.0, 0.0)),
    dict(x_boundary=1, inlet_kind=1, inlet_density=0.0),
    dict(x_boundary=1, outlet_density=-1.0),
])
def test_create_rejects_bad_params_before_device(bad):
    kw = dict(nx=32, ny=32, nz=32, tau=0.8)
    kw.update(bad)
    with pytest.raises(dilbm.DilbmError) as e:
        dilbm3d.Solver3D(dilbm3d.Params3D(**kw))
    assert e.value.status == dilbm.EINVAL


def test_abi_version_mismatch():
    lib = dilbm3d.load()
    p = dilbm3d.Params3D(nx=8, ny=8, nz=8, tau=0.8).to_c()
    p.abi_version = 99
    h = C.c_void_p()
    assert lib.dilbm3d_create(C.byref(p), C.byref(h)) == dilbm.EABI
    assert not h.value
    assert b"abi" in lib.dilbm3d_last_error(None)


def test_null_handles_are_rejected():
    lib = dilbm3d.load()
    assert lib.dilbm3d_step(None, 1) == dilbm.EINVAL
    assert lib.dilbm3d_get_fields(None, None, None, None, None) == dilbm.EINVAL
    assert lib.dilbm3d_set_populations(None, None) == dilbm.EINVAL
    assert lib.dilbm3d_get_wall_force(None, None) == dilbm.EINVAL
    lib.dilbm3d_destroy(None)
    assert lib.dilbm3d_create(None, None) == dilbm.EINVAL


def test_batch_rejects_bad_arguments_before_device():
    lib = dilbm3d.load()
    h = C.c_void_p()
    assert lib.dilbm3d_batch_create(None, 0, C.byref(h)) == dilbm.EINVAL and not h.value
    arr = (C.c_void_p * 2)(None, None)
    assert lib.dilbm3d_batch_create(arr, 2, C.byref(h)) == dilbm.EINVAL and not h.value
    assert lib.dilbm3d_batch_last_error(None) == b"NULL member"
    assert lib.dilbm3d_batch_create(arr, 2, None) == dilbm.EINVAL
    assert lib.dilbm3d_batch_step(None, 1) == dilbm.EINVAL
    lib.dilbm3d_batch_destroy(None)  # a no-op
