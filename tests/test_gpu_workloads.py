"""GPU parity on the benchmark workloads, at full size, plus the maximum lattice size, FP16
storage and the error paths.

Tolerances, fixed before measuring:
* FP32 storage: velocity relative L2 <= 1e-5 after 1000 steps, body positions within
  1e-4 lattice units;
* FP16 storage: velocity relative L2 <= 2e-3, positions within 1e-2;
* one step from the same state: populations within 256 * 2^-24 of the largest deviation
  (FP32), as in test_gpu_parity.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2106_08950_amd import dilbm, inputs
from helpers import gpu_solver, log_case, oracle_solver, velocity_rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
U32 = 2.0**-24


def _golden(name, wl):
    from make_golden import workload_digest

    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} has not been generated (tests/golden/make_golden.py)")
    g = np.load(path)
    assert json.loads(str(g["meta"]))["digest"] == workload_digest(wl), "inputs changed"
    return g


def _wrap_err(a, b, n):
    d = np.abs(np.asarray(a) - np.asarray(b))
    return np.minimum(d, np.asarray(n) - d)


def test_settling_disc_trajectory_fp32():
    wl = inputs.settling_disc()
    gold = _golden("settling_disc.npz", wl)
    traj = gold["traj"]
    every = int(traj[1, 0] - traj[0, 0])
    log_case("settling disc 400x1600, 20000 steps, FP32")
    g = gpu_solver(wl)
    errs = []
    for k in range(1, len(traj)):
        g.step(every)
        x, u, om = g.get_particles()
        errs.append(np.abs(x[0] - traj[k, 1:3]).max())
        if k * every == 1000:
            rho, ux, uy = g.get_fields()
            e = velocity_rel_l2(ux[::8, ::8], uy[::8, ::8], gold["ux_1000_s8"], gold["uy_1000_s8"])
            assert e <= 1e-5, e
    print(f"settling FP32: max position error over 20000 steps {max(errs):.3e}")
    assert max(errs) <= 1e-4
    x, u, om = g.get_particles()
    assert abs(u[0, 1] - traj[-1, 4]) <= 1e-4 * abs(traj[-1, 4])


def test_settling_disc_trajectory_fp16():
    wl = inputs.settling_disc()
    gold = _golden("settling_disc.npz", wl)
    traj = gold["traj"]
    every = int(traj[1, 0] - traj[0, 0])
    log_case("settling disc 400x1600, 20000 steps, FP16")
    g = gpu_solver(wl, storage=dilbm.STORE_FP16)
    errs = []
    for k in range(1, len(traj)):
        g.step(every)
        x, u, om = g.get_particles()
        errs.append(np.abs(x[0] - traj[k, 1:3]).max())
        if k * every == 1000:
            rho, ux, uy = g.get_fields()
            e = velocity_rel_l2(ux[::8, ::8], uy[::8, ::8], gold["ux_1000_s8"], gold["uy_1000_s8"])
            print(f"settling FP16: u rel L2 at 1000 steps {e:.3e}")
            assert e <= 2e-3, e
    print(f"settling FP16: max position error over 20000 steps {max(errs):.3e}")
    assert max(errs) <= 1e-2


def test_cylinder_channel_fp16():
    wl = inputs.cylinder_channel()
    gold = _golden("cylinder_channel.npz", wl)
    log_case("cylinder channel FP16 1000 steps")
    g = gpu_solver(wl, storage=dilbm.STORE_FP16)
    g.step(1000)
    rho, ux, uy = g.get_fields()
    e = velocity_rel_l2(ux, uy, gold["ux_1000"], gold["uy_1000"])
    print(f"cylinder FP16: u rel L2 at 1000 steps {e:.3e}")
    assert e <= 2e-3


@pytest.mark.parametrize("storage", [dilbm.STORE_FP32, dilbm.STORE_FP16])
def test_dense_suspension_1000_steps(storage):
    wl = inputs.dense_suspension()
    gold = _golden("dense_suspension_1000.npz", wl)
    log_case(f"dense suspension 4096^2, 2000 discs, 1000 steps, storage={storage}")
    g = gpu_solver(wl, storage=storage)
    g.step(1000)
    x, u, om = g.get_particles()
    rho, ux, uy = g.get_fields()
    pos_err = _wrap_err(x, gold["pos"], [wl.nx, wl.ny]).max()
    # the velocity on 16 full rows, 16 full columns and two 128 x 128 windows around discs
    # (every node of each), and on every 32nd node in both directions
    rows, cols, wins = gold["rows"], gold["cols"], gold["wins"]
    w = int(gold["u_wins"].shape[-1])
    g_parts = [np.stack([ux[rows], uy[rows]]).ravel(), np.stack([ux[:, cols], uy[:, cols]]).ravel()]
    o_parts = [gold["u_rows"].ravel(), gold["u_cols"].ravel()]
    for k, (x0, y0) in enumerate(wins):
        g_parts.append(np.stack([ux[y0:y0 + w, x0:x0 + w], uy[y0:y0 + w, x0:x0 + w]]).ravel())
        o_parts.append(gold["u_wins"][k].ravel())
    gs, os_ = np.concatenate(g_parts), np.concatenate(o_parts).astype(np.float64)
    u_err = float(np.linalg.norm(gs - os_) / np.linalg.norm(os_))
    u_err_s32 = velocity_rel_l2(ux[::32, ::32], uy[::32, ::32], gold["ux_s32"], gold["uy_s32"])
    vel_err = np.abs(u - gold["vel"]).max() / np.abs(gold["vel"]).max()
    print(f"suspension storage={storage}: position error {pos_err:.3e}, u rel L2 (rows, "
          f"columns, windows) {u_err:.3e}, every 32nd node {u_err_s32:.3e}, body velocity rel "
          f"error {vel_err:.3e}")
    if storage == dilbm.STORE_FP32:
        assert pos_err <= 1e-4 and u_err <= 1e-5 and u_err_s32 <= 1e-5
    else:
        assert pos_err <= 1e-2 and u_err <= 2e-3 and u_err_s32 <= 2e-3


def test_dense_suspension_one_step_full_size():
    # one step from a seeded random state at the benchmark size, every population compared
    wl = inputs.dense_suspension()
    f0 = inputs.random_deviations(wl.nx, wl.ny, amp=1e-4, seed=33)
    log_case("dense suspension 4096^2 one step, full comparison")
    g = gpu_solver(wl)
    g.set_populations(f0)
    g.step(1)
    fg = g.get_populations()
    Fg, Tg = g.get_particle_forces()
    xg, ug, wg = g.get_particles()
    g.close()
    o = oracle_solver(wl)
    o.set_populations(f0)
    del f0
    o.step(1)
    fo = o.get_populations()
    err = np.abs(fg - fo).max() / np.abs(fo).max()
    del fg, fo
    assert err <= 256 * U32, err
    Fo, To = o.get_particle_forces()
    assert np.abs(Fg - Fo).max() <= 1e-4 * np.abs(Fo).max()
    assert np.abs(Tg - To).max() <= 1e-4 * np.abs(To).max()
    xo, uo, wo = o.get_particles()
    assert _wrap_err(xg, xo, [wl.nx, wl.ny]).max() < 1e-9


def _check_by_windows(g, nx, ny, steps, G, discs, R, rho_s, W=96, tol=1e-5, far=8):
    """A solve started from rest under a body force G, advanced `steps` steps: nodes
    farther than the support plus `steps` from every disc are untouched by them and have
    u = (n + 1/2) G; the neighbourhood of each disc equals a small periodic oracle solve
    holding the same disc at the same place relative to its window (stitched across the
    periodic seams)."""
    xg, ug, wg = g.get_particles()
    Fg, Tg = g.get_particle_forces()
    rng = np.random.default_rng(1)
    for _ in range(far):
        while True:
            x0 = int(rng.integers(0, nx - 8))
            y0 = int(rng.integers(0, ny - 8))
            d = np.abs(np.asarray(discs) - [x0 + 4, y0 + 4])
            d = np.minimum(d, [nx, ny] - d)
            if np.all(np.hypot(d[:, 0], d[:, 1]) > R + 8 + steps + 16):
                break
        rho, ux, uy = g.get_fields_region(x0, y0, 8, 8)
        if tol <= 1e-5:  # FP32: every node
            assert np.allclose(ux, (steps + 0.5) * G[0], rtol=1e-5, atol=0)
            assert np.allclose(uy, (steps + 0.5) * G[1], rtol=1e-5, atol=0)
        else:  # FP16: relative L2 over the 8 x 8 window
            e = velocity_rel_l2(ux, uy, np.full_like(ux, (steps + 0.5) * G[0]),
                                np.full_like(uy, (steps + 0.5) * G[1]))
            assert e <= tol, e
    h = W // 2
    for b in range(len(discs)):
        cx, cy = int(np.floor(discs[b][0])), int(np.floor(discs[b][1]))
        ox, oy = cx - h, cy - h   # window origin (may be negative or past the end: wraps)
        ux_w = np.empty((W, W))
        uy_w = np.empty((W, W))
        for j in range(W):
            yy = (oy + j) % ny
            # split the row at the x seam
            xs = [(ox + i) % nx for i in range(W)]
            i = 0
            while i < W:
                run = 1
                while i + run < W and xs[i + run] == xs[i] + run:
                    run += 1
                _, a, c = g.get_fields_region(xs[i], yy, run, 1)
                ux_w[j, i:i + run] = a[0]
                uy_w[j, i:i + run] = c[0]
                i += run
        small = inputs.Workload(name="win", nx=W, ny=W, tau=0.8, nsteps=steps, G=G,
                                **inputs._bodies([[discs[b][0] - ox, discs[b][1] - oy]], [R],
                                                 [rho_s]))
        o = oracle_solver(small)
        o.step(steps)
        ro, uxo, uyo = o.get_fields()
        err = velocity_rel_l2(ux_w, uy_w, uxo, uyo)
        assert err < tol, (b, err)
        xo, uo, wo = o.get_particles()
        assert np.abs((xg[b] - [ox, oy]) % [nx, ny] - xo[0]).max() < 1e-9
        Fo, To = o.get_particle_forces()
        assert np.abs(Fg[b] - Fo[0]).max() <= max(tol, 1e-4) * np.abs(Fo[0]).max()


@pytest.mark.parametrize("storage,nx,ny,tile", [
    (dilbm.STORE_FP32, 8192, 8192, -1),   # 2.4 GB per population buffer: 32-bit plane offsets
    (dilbm.STORE_FP32, 8192, 8192, 0),    # the same with 64 x 4 tiles (chunked order)
    (dilbm.STORE_FP16, 16384, 8192, -1),  # FP16, 2.4 GB per buffer
])
def test_plane_offset_addressing_by_windows(storage, nx, ny, tile):
    """Lattices whose population buffer passes 2 GB but whose planes stay under it take the
    collide instances with a scalar plane base and 32-bit offsets.  Discs across both
    periodic seams and at large coordinates; 4 steps from rest under a body force, checked
    far from the discs and by windows around each."""
    steps = 4
    G = (1e-5, 2e-6)
    discs = [[nx - 2.7, ny - 3.4], [nx - 5000.3, ny - 1000.6], [3.2, 4100.7]]
    R, rho_s = 6.0, 1.3
    wl = inputs.Workload(name="g32", nx=nx, ny=ny, tau=0.8, nsteps=steps, G=G,
                         **inputs._bodies(discs, [R] * 3, [rho_s] * 3))
    log_case(f"plane-offset addressing {nx}x{ny} storage={storage} tile={tile}")
    g = gpu_solver(wl, storage=storage, tile=tile)
    g.step(steps)
    _check_by_windows(g, nx, ny, steps, G, discs, R, rho_s,
                      tol=1e-5 if storage == dilbm.STORE_FP32 else 2e-3)
    g.close()


def test_maximum_lattice_size_by_windows():
    """nx * ny just below 2^31 (65536 x 32767, 155 GB of FP32 populations): a disc across
    both periodic seams and one at large coordinates, 4 steps from rest under a body
    force.  Nodes farther than the support plus 4 steps are untouched by the discs and
    have u = (n + 1/2) G exactly; the neighbourhood of each disc equals a small periodic
    oracle solve holding the same disc at the same place relative to its window."""
    nx, ny, steps = 65536, 32767, 4
    G = (1e-5, 2e-6)
    discs = [[nx - 2.7, ny - 3.4], [40000.3, 20000.6]]
    R, rho_s = 6.0, 1.3
    wl = inputs.Workload(name="max", nx=nx, ny=ny, tau=0.8, nsteps=steps, G=G,
                         **inputs._bodies(discs, [R, R], [rho_s, rho_s]))
    log_case("maximum lattice 65536x32767 FP32 (155 GB)")
    g = gpu_solver(wl)
    g.step(steps)
    _check_by_windows(g, nx, ny, steps, G, discs, R, rho_s)
    g.close()


@pytest.mark.parametrize("cap,tile", [(1, 0), (2, 0), (2, 2)])
def test_lists_filled_to_capacity_match_oracle(cap, tile):
    """Lists exactly as long as the bodies need.  With capacity 1 every entry sits in the
    tiles' heads; with 2, the tiles the two bodies share hold their second entry in the
    list array."""
    pos = [[30.0, 32.0]] if cap == 1 else [[22.0, 32.0], [40.0, 33.5]]
    vel = [[0.01, 0.004]] if cap == 1 else [[0.01, 0.0], [-0.005, 0.006]]
    wl = inputs.Workload(name="cap_exact", nx=96, ny=64, tau=0.7, nsteps=200, G=(1e-5, 0.0),
                         **inputs._bodies(pos, [5.0] * len(pos), [1.3] * len(pos), vel=vel))
    log_case(f"lists filled to capacity {cap}, tile shape {tile}, 200 steps")
    g = gpu_solver(wl, list_capacity=cap, tile=tile)
    o = oracle_solver(wl)
    g.step(200)
    o.step(200)
    _, ux, uy = g.get_fields()
    _, uxo, uyo = o.get_fields()
    assert velocity_rel_l2(ux, uy, uxo, uyo) < 1e-5
    xg, _, _ = g.get_particles()
    xo, _, _ = o.get_particles()
    assert np.abs(xg - xo).max() < 1e-4
    g.close()


def test_capacity_overflow_poisons_handle():
    wl = inputs.Workload(name="cap", nx=64, ny=64, tau=0.8, nsteps=1,
                         **inputs._bodies([[30.0, 30.0], [34.0, 31.0], [20.0, 40.0]],
                                          [5.0, 5.0, 4.0], [1.2, 1.2, 1.2]))
    log_case("capacity overflow")
    g = dilbm.Solver(dilbm.params_from_workload(wl, list_capacity=1))
    with pytest.raises(dilbm.DilbmError) as e:
        g.set_particles(wl.pos, wl.radius, wl.density)
    assert e.value.status == dilbm.ECAPACITY
    with pytest.raises(dilbm.DilbmError) as e:
        g.step(1)
    assert e.value.status == dilbm.ESTATE
    x, u, om = g.get_particles()  # reads still work
    assert x.shape == (3, 2)
    g.close()


def test_blow_up_is_reported_and_poisons_handle():
    wl = inputs.Workload(name="blow", nx=32, ny=32, tau=0.500001, nsteps=1, G=(0.1, 0.0),
                         **inputs._bodies([[16.0, 16.0]], [4.0], [1.2]))
    log_case("forced blow-up")
    g = gpu_solver(wl)
    with pytest.raises(dilbm.DilbmError) as e:
        g.step(50)
    assert e.value.status == dilbm.EUNSTABLE
    with pytest.raises(dilbm.DilbmError) as e:
        g.step(1)
    assert e.value.status == dilbm.ESTATE
    rho, ux, uy = g.get_fields()
    assert rho.shape == (32, 32)
    g.close()


def test_failure_stops_a_long_call_within_two_chunks():
    """Uniform acceleration G = 1e-3 drives |u| past 0.5 at step 500: a call of 4000 steps
    (32-step graph chunks) stops within two chunks of the failure and returns the error."""
    wl = inputs.Workload(name="blowup", nx=64, ny=48, tau=0.8, nsteps=1, G=(1e-3, 0.0))
    log_case("blow-up in a long call")
    g = gpu_solver(wl)
    assert g.step_status(4000) == dilbm.EUNSTABLE
    n = g.step_count()
    assert 500 < n <= 501 + 2 * 32, n
    assert g.step_status(1) == dilbm.ESTATE
    g.close()


def test_set_particles_between_steps_and_empty_body_set():
    wl, f0 = inputs.cylinder_channel(), None
    log_case("set_particles between steps")
    g = gpu_solver(wl)
    o = oracle_solver(wl)
    g.step(50)
    o.step(50)
    rng = np.random.default_rng(3)
    b = inputs.random_bodies(rng, wl.nx, wl.ny, 4, rmin=3, rmax=6)
    g.set_particles(b["pos"], b["radius"], b["density"], b["vel"], b["omega"], b["fixed"])
    o.set_particles(b["pos"], b["radius"], b["density"], b["vel"], b["omega"], b["fixed"])
    F, T = g.get_particle_forces()
    assert np.all(F == 0) and np.all(T == 0)  # no step since the new body set
    g.step(50)
    o.step(50)
    g.set_particles(np.zeros((0, 2)), np.zeros(0), np.zeros(0))
    o.set_particles(np.zeros((0, 2)), np.zeros(0), np.zeros(0))
    g.step(20)
    o.step(20)
    _, uxg, uyg = g.get_fields()
    _, uxo, uyo = o.get_fields()
    assert velocity_rel_l2(uxg, uyg, uxo, uyo) < 1e-5
    assert g.step_count() == 120
