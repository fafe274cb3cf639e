"""Write the stored expected values of the long parity cases.

Every value written here comes from the FP64 oracle (``oracle/``) run on the seeded
inputs of ``paper_2106_08950_amd.inputs``; nothing comes from the GPU library.  Each file
also records a digest of its inputs, so a test can tell when the generator has changed.

    python tests/golden/make_golden.py cylinder   # 200x80 channel, 2000 steps  (~1 min)
    python tests/golden/make_golden.py settling   # 400x1600 box, 20000 steps   (~20 min)
    python tests/golden/make_golden.py suspension # 4096^2, 2000 discs, 1000 steps (~10 min)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2106_08950_amd import inputs  # noqa: E402


def workload_digest(wl) -> str:
    h = hashlib.sha256()
    scalars = (wl.nx, wl.ny, wl.tau, wl.rho0, wl.eps, wl.cutoff, tuple(wl.G), tuple(wl.g),
               wl.wall_mask, wl.wall_h, wl.force_mode, wl.eps_p, wl.eps_p1, wl.eps_w,
               wl.eps_w1, wl.xi)
    h.update(repr(scalars).encode())
    for a in (wl.pos, wl.vel, wl.omega, wl.radius, wl.density):
        h.update(np.ascontiguousarray(a, np.float64).tobytes())
    h.update(np.ascontiguousarray(wl.fixed, np.uint8).tobytes())
    return h.hexdigest()


def solver_for(wl):
    p = oracle.OracleParams(nx=wl.nx, ny=wl.ny, tau=wl.tau, rho0=wl.rho0, eps=wl.eps,
                            cutoff=wl.cutoff, G=tuple(wl.G), g=tuple(wl.g),
                            wall_mask=wl.wall_mask, wall_h=wl.wall_h, force_mode=wl.force_mode,
                            eps_p=wl.eps_p, eps_p1=wl.eps_p1, eps_w=wl.eps_w, eps_w1=wl.eps_w1,
                            xi=wl.xi)
    s = oracle.OracleSolver(p)
    if wl.nbodies:
        s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    return s


def _meta(wl, extra):
    return json.dumps({"workload": wl.name, "digest": workload_digest(wl),
                       "oracle_threads": oracle.num_threads(), **extra})


def cylinder():
    wl = inputs.cylinder_channel()
    s = solver_for(wl)
    forces = np.zeros((wl.nsteps, 3))
    wall = np.zeros((wl.nsteps, 2))
    out = {}
    t0 = time.time()
    for n in range(1, wl.nsteps + 1):
        s.step(1)
        F, T = s.get_particle_forces()
        forces[n - 1] = (F[0, 0], F[0, 1], T[0])
        wall[n - 1] = s.get_wall_force()
        if n in (1000, 2000):
            rho, ux, uy = s.get_fields()
            out[f"rho_{n}"] = rho
            out[f"ux_{n}"] = ux
            out[f"uy_{n}"] = uy
    np.savez_compressed(os.path.join(HERE, "cylinder_channel.npz"), forces=forces, wall=wall,
                        meta=_meta(wl, {"seconds": time.time() - t0}), **out)


def settling():
    wl = inputs.settling_disc()
    s = solver_for(wl)
    every = 100
    traj = np.zeros((wl.nsteps // every + 1, 8))  # step, x, y, ux, uy, omega, Fx, Fy
    x, u, om = s.get_particles()
    traj[0] = (0, x[0, 0], x[0, 1], u[0, 0], u[0, 1], om[0], 0, 0)
    out = {}
    t0 = time.time()
    for k in range(1, wl.nsteps // every + 1):
        s.step(every)
        x, u, om = s.get_particles()
        F, T = s.get_particle_forces()
        traj[k] = (k * every, x[0, 0], x[0, 1], u[0, 0], u[0, 1], om[0], F[0, 0], F[0, 1])
        if k * every == 1000:
            rho, ux, uy = s.get_fields()
            out["ux_1000_s8"] = ux[::8, ::8].copy()
            out["uy_1000_s8"] = uy[::8, ::8].copy()
        print(f"settling step {k * every} y={x[0, 1]:.4f} v={u[0, 1]:.3e} "
              f"{time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(os.path.join(HERE, "settling_disc.npz"), traj=traj,
                        meta=_meta(wl, {"seconds": time.time() - t0, "every": every}), **out)


def suspension():
    wl = inputs.dense_suspension()
    s = solver_for(wl)
    steps = 1000
    t0 = time.time()
    for k in range(10):
        s.step(steps // 10)
        print(f"suspension step {(k + 1) * steps // 10} {time.time() - t0:.0f}s", flush=True)
    x, u, om = s.get_particles()
    F, T = s.get_particle_forces()
    rho, ux, uy = s.get_fields()
    rows, cols, wins = suspension_sample(wl)
    win = np.stack([np.stack([ux[y0:y0 + WIN, x0:x0 + WIN], uy[y0:y0 + WIN, x0:x0 + WIN]])
                    for x0, y0 in wins])
    np.savez_compressed(os.path.join(HERE, "dense_suspension_1000.npz"), pos=x, vel=u, omega=om,
                        force=F, torque=T, ux_s32=ux[::32, ::32].copy(),
                        uy_s32=uy[::32, ::32].copy(), rho_s32=rho[::32, ::32].copy(),
                        ux_norm=np.linalg.norm(np.stack([ux, uy])),
                        # full rows and columns and two windows around discs, in FP32 (its
                        # round-off, 6e-8 relative, is far below the 1e-5 bound)
                        u_rows=np.stack([ux[rows], uy[rows]]).astype(np.float32),
                        u_cols=np.stack([ux[:, cols], uy[:, cols]]).astype(np.float32),
                        u_wins=win.astype(np.float32), rows=rows, cols=cols,
                        wins=np.asarray(wins),
                        meta=_meta(wl, {"seconds": time.time() - t0, "steps": steps}))


WIN = 128


def suspension_sample(wl):
    """Where the 1000-step suspension velocity is stored: 16 full rows and 16 full columns
    spread over the lattice, and two WIN x WIN windows centred on the first two discs'
    starting positions (kept inside the lattice)."""
    rows = (np.arange(16) * (wl.ny // 16) + 37) % wl.ny
    cols = (np.arange(16) * (wl.nx // 16) + 101) % wl.nx
    wins = []
    for b in range(2):
        x0 = int(np.clip(np.floor(wl.pos[b, 0]) - WIN // 2, 0, wl.nx - WIN))
        y0 = int(np.clip(np.floor(wl.pos[b, 1]) - WIN // 2, 0, wl.ny - WIN))
        wins.append((x0, y0))
    return rows, cols, wins


if __name__ == "__main__":
    oracle.build_oracle(force=False)
    for name in sys.argv[1:]:
        {"cylinder": cylinder, "settling": settling, "suspension": suspension}[name]()
