"""The C ABI on the CPU: the library loads, exports every symbol include/dilbm.h
declares, and rejects bad arguments before touching a device (no compute calls)."""
import ctypes as C
import os
import re

import pytest

from paper_2106_08950_amd import dilbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dilbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dilbm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_what_the_binding_knows():
    assert _declared() == sorted(dilbm.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = dilbm.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_params_struct_layout_round_trips():
    lib = dilbm.load()
    p = dilbm.dilbm_params()
    lib.dilbm_params_init(C.byref(p))
    assert p.abi_version == dilbm.ABI_VERSION
    assert (p.tau, p.rho0, p.interface_width, p.phi_cutoff) == (0.8, 1.0, 2.0, 4.0)
    assert (p.coll_eps_p, p.coll_eps_w, p.coll_xi) == (1.0e4, 0.5e4, 1.0)
    assert (p.storage, p.list_capacity, p.tile, p.device) == (0, 0, -1, 0)
    assert p.fp16_scale_log2 == dilbm.FP16_SCALE_AUTO == -1
    assert p.stream is None


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(nx=70000), dict(tau=0.5), dict(tau=float("nan")),
    dict(rho0=0.0), dict(interface_width=0.0), dict(phi_cutoff=-1.0), dict(wall_mask=4),
    dict(wall_mask=1, wall_half_thickness=0.0), dict(force_mode=2), dict(storage=3),
    dict(fp16_scale_log2=30), dict(fp16_scale_log2=-2), dict(list_capacity=5000), dict(tile=9), dict(coll_xi=-1.0),
    dict(body_force=(float("inf"), 0.0)),
])
def test_create_rejects_bad_params_before_device(bad):
    kw = dict(nx=32, ny=32)
    kw.update(bad)
    with pytest.raises(dilbm.DilbmError) as e:
        dilbm.Solver(dilbm.Params(**kw))
    assert e.value.status == dilbm.EINVAL


def test_abi_version_mismatch():
    lib = dilbm.load()
    p = dilbm.Params(nx=8, ny=8).to_c()
    p.abi_version = 99
    h = C.c_void_p()
    assert lib.dilbm_create(C.byref(p), C.byref(h)) == dilbm.EABI
    assert not h.value
    assert b"abi" in lib.dilbm_last_error(None)


def test_null_handles_are_rejected():
    lib = dilbm.load()
    assert lib.dilbm_step(None, 1) == dilbm.EINVAL
    assert lib.dilbm_get_fields(None, None, None, None) == dilbm.EINVAL
    assert lib.dilbm_pool_run(None, 1) == dilbm.EINVAL
    lib.dilbm_destroy(None)
    lib.dilbm_pool_destroy(None)
    assert lib.dilbm_create(None, None) == dilbm.EINVAL


def test_footprint_counts_populations_and_bodies():
    p = dilbm.Params(nx=4096, ny=4096)
    fp32 = dilbm.footprint(p, 2000)
    assert fp32 >= 2 * 9 * 4096 * 4096 * 4
    p16 = dilbm.Params(nx=4096, ny=4096, storage=dilbm.STORE_FP16)
    fp16 = dilbm.footprint(p16, 2000)
    assert fp32 - fp16 == 2 * 9 * 4096 * 4096 * 2
    assert dilbm.footprint(p, 10) < fp32


def test_tile_shapes_cover_256_nodes():
    shapes = dilbm.tile_shapes()
    assert len(shapes) == 6
    assert all(tx * ty == 256 for tx, ty in shapes[:5])
    assert shapes[5] == (512, 1)  # two nodes per lane


def test_pair_tile_shape_needs_fp16_and_even_width():
    bad = [dict(nx=1024, ny=8, tile=5), dict(nx=1023, ny=8, tile=5, storage=dilbm.STORE_FP16)]
    for kw in bad:
        with pytest.raises(dilbm.DilbmError) as e:
            dilbm.footprint(dilbm.Params(**kw), 0)
        assert e.value.status == dilbm.EINVAL
    assert dilbm.footprint(dilbm.Params(nx=1024, ny=8, tile=5, storage=dilbm.STORE_FP16), 0) > 0


def test_one_hip_runtime_per_process():
    """The library binds to the HIP runtime PyTorch already holds: a process that also
    uses torch streams and tensors must not map a second copy of the runtime."""
    dilbm.load()
    with open("/proc/self/maps") as f:
        paths = {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    assert len(paths) == 1, paths


@pytest.mark.parametrize("bad", [
    dict(x_boundary=2),
    dict(x_boundary=1, nx=2),
    dict(x_boundary=1, wall_mask=2),
    dict(x_boundary=1, inlet_kind=2),
    dict(x_boundary=1, outlet_kind=3),
    dict(x_boundary=1, inlet_profile=2),
    dict(x_boundary=1, inlet_kind=1, inlet_density=0.0),
    dict(x_boundary=1, outlet_kind=0, outlet_density=-1.0),
    dict(x_boundary=1, inlet_velocity=(float("nan"), 0.0)),
])
def test_create_rejects_bad_open_ends_before_device(bad):
    base = dict(nx=32, ny=16)
    base.update(bad)
    p = dilbm.Params(**base)
    h = C.c_void_p()
    st = dilbm.load().dilbm_create(C.byref(p.to_c()), C.byref(h))
    assert st == dilbm.EINVAL and not h.value
