"""Benchmark of the DI-LBM time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage fp32|fp16] [--no-cpu]

Workload (one step = the whole hot path over one solve): the dense suspension of
4096 x 4096 periodic nodes with 2000 free discs of radius 8 (seed 3), tau = 0.6, body
force 1e-6, FP32 shifted-population storage -- its 1.2 GB working set exceeds the
256 MB Infinity Cache, so the populations stream from HBM every step.  Inputs are
resident in HBM before the timed region starts.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, FP32 vs batched/FP16; p50/p99 latency of served solves"
HBM_PEAK_GBS = 8000.0


def run_oracle_sample(wl, steps):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    import oracle

    oracle.build_oracle(force=False)
    p = oracle.OracleParams(nx=wl.nx, ny=wl.ny, tau=wl.tau, rho0=wl.rho0, eps=wl.eps,
                            cutoff=wl.cutoff, G=tuple(wl.G), g=tuple(wl.g),
                            wall_mask=wl.wall_mask, wall_h=wl.wall_h, force_mode=wl.force_mode)
    s = oracle.OracleSolver(p)
    s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    s.step(1)  # warm
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    s.close()
    return {"value": round(wl.nodes * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{wl.name}: {steps} steps after 1 warm-up step, FP64, "
                      f"{oracle.num_threads()} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", choices=["fp32", "fp16"], default="fp32")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the slab decomposition is described in DESIGN.md); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2106_08950_amd import dilbm, inputs

    torch.cuda.init()
    wl = inputs.dense_suspension()
    storage = dilbm.STORE_FP16 if args.storage == "fp16" else dilbm.STORE_FP32
    stream = torch.cuda.Stream()
    prm = dilbm.params_from_workload(wl, storage=storage, tile=args.tile, device=0,
                                     stream=stream.cuda_stream)
    s = dilbm.Solver(prm)
    s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    s.step(args.warmup)

    s.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    collide_ms, launches = s.kernel_timing()
    s.set_kernel_timing(False)

    nodes = wl.nodes
    mlups = nodes * args.steps / dt / 1e6
    bytes_per_node = 72 if storage == dilbm.STORE_FP32 else 36
    avg_ms = collide_ms / max(launches, 1)
    achieved = bytes_per_node * nodes / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "bodies": wl.nbodies,
                   "tau": wl.tau, "storage": args.storage, "tile": prm.tile},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "kernel": "k_collide", "bytes_per_node": bytes_per_node,
                     "avg_launch_ms": round(avg_ms, 5), "launches": launches},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = run_oracle_sample(wl, args.cpu_steps)
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
