"""dilbm_get_fields_region_noalloc (the entry point for callers that cannot allocate)
against dilbm_get_fields_region on the same state, through the C ABI: two calls in a row,
the second on a smaller region, both bitwise equal to the allocating call (the same
kernel reads the same populations); regions beyond the fixed staging array are refused."""
import numpy as np
import pytest

from paper_2106_08950_amd import dilbm, inputs
from helpers import gpu_solver, log_case

pytestmark = pytest.mark.gpu


def _case():
    rng = np.random.default_rng(17)
    b = inputs.random_bodies(rng, 1100, 1060, 12, rmin=4.0, rmax=9.0)
    wl = inputs.Workload(name="noalloc", nx=1100, ny=1060, tau=0.7, nsteps=30,
                         G=(1e-5, -2e-6), wall_mask=inputs.WALL_Y, wall_h=3.0, **b)
    return wl


@pytest.mark.parametrize("storage", [dilbm.STORE_FP32, dilbm.STORE_FP16])
def test_noalloc_fields_equal_the_allocating_call(storage):
    wl = _case()
    log_case(f"no-alloc field readback, storage={storage}")
    g = gpu_solver(wl, storage=storage)
    g.step(wl.nsteps)
    # first call: the largest region the staging array takes (1024 x 1024 = 2^20 nodes)
    for (x0, y0, w, h) in [(30, 0, 1024, 1024), (517, 333, 77, 45)]:
        ref = g.get_fields_region(x0, y0, w, h)
        got = g.get_fields_region_noalloc(x0, y0, w, h)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert np.abs(got[1]).max() > 0
    # after more steps, a third region: the array keeps no stale values
    g.step(5)
    ref = g.get_fields_region(0, 1050, 1100, 10)
    got = g.get_fields_region_noalloc(0, 1050, 1100, 10)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    # beyond the staging array: refused, the handle stays usable
    with pytest.raises(dilbm.DilbmError) as e:
        g.get_fields_region_noalloc(0, 0, 1025, 1024)
    assert e.value.status == dilbm.EINVAL
    with pytest.raises(dilbm.DilbmError) as e:
        g.get_fields_region_noalloc(1000, 0, 101, 10)  # outside the lattice
    assert e.value.status == dilbm.EINVAL
    g.step(1)
    g.close()


def test_noalloc_fields_two_handles_one_after_another():
    wl = _case()
    log_case("no-alloc field readback, two handles")
    a = gpu_solver(wl)
    b = gpu_solver(inputs.Workload(**{**wl.__dict__, "G": (-2e-5, 1e-5)}))
    a.step(10)
    b.step(10)
    ra = a.get_fields_region_noalloc(100, 100, 300, 200)
    rb = b.get_fields_region_noalloc(100, 100, 300, 200)
    for x, y in zip(ra, a.get_fields_region(100, 100, 300, 200)):
        assert np.array_equal(x, y)
    for x, y in zip(rb, b.get_fields_region(100, 100, 300, 200)):
        assert np.array_equal(x, y)
    assert not np.array_equal(ra[1], rb[1])
    a.close()
    b.close()
