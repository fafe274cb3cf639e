"""Benchmark of the DI-LBM time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--legs fp32,fp16,open_ends,suspension3d,batched,served]
                    [--no-cpu]

Headline workload (one step = the whole hot path over one solve): the dense suspension of
4096 x 4096 periodic nodes with 2000 free discs of radius 8 (seed 3), tau = 0.6, body
force 1e-6, FP32 shifted-population storage -- its 1.2 GB working set exceeds the 256 MB
Infinity Cache, so the populations stream from HBM every step.  Inputs are resident in
HBM before the timed region starts.  Further legs, reported in the same JSON line:
* fp16: the same workload with FP16 storage (36 B per node update);
* open_ends: a 4096 x 2048 inflow channel (velocity inlet, zero-gradient outlet, 300
  fixed discs), FP32;
* suspension3d: the three-dimensional path, 256^3 D3Q19 nodes with 400 free spheres
  (seed 8), FP32 (152 B per node update);
* batched: the 256-solve ensemble (2000 steps each) advanced as one pool, against the
  same solves run one after another as plain solves;
* served: the 500-request Poisson stream (50 requests/s) through the continuous-batching
  loop, with p50/p99 completion latency.
Prints one JSON line.
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
KERNEL_SRC = os.path.join(ROOT, "paper_2106_08950_amd", "csrc", "kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "k_collide_dense_suspension_4096_fp32_hbm_counters.txt")
KERNEL3_SRC = os.path.join(ROOT, "paper_2106_08950_amd", "csrc", "kernels3d.hip")
COUNTERS3 = os.path.join(ROOT, "profiles", "k3_collide_suspension3d_256_fp32_hbm_counters.txt")
COUNTERS16 = os.path.join(ROOT, "profiles", "k_collide_dense_suspension_4096_fp16_hbm_counters.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(src=None):
    import hashlib

    with open(src or KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(counters=None, src=None):
    """HBM bytes per collide launch from a committed rocprofv3 counter summary (default:
    the 2-D headline's), or None when the kernel source has changed since the counters
    were taken."""
    try:
        with open(counters or COUNTERS) as f:
            kv = dict(ln.split(":", 1) for ln in f.read().splitlines() if ":" in ln)
    except OSError:
        return None
    if kv.get("kernel_source_sha256_16", "").strip() != kernel_source_hash(src):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain 1 GiB device copy, three times: the known traffic that the FETCH_SIZE and
    WRITE_SIZE counters are scaled by."""
    import torch

    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB (read 1 GiB + write 1 GiB per copy)", flush=True)


def copy_reference(nbytes):
    """A plain device-to-device copy of the population volume (nbytes read, nbytes
    written), timed with events: the second denominator of the roofline."""
    import torch

    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    reps = 20
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return 2 * n * 4 / (ms * 1e-3) / 1e9


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
                      f"{oracle.num_threads()} OpenMP threads, {dt:.1f} s"}


def single_solve(wl, storage, steps, warmup, tile, stream):
    """Timed single-solve run; returns (mlups, seconds, collide_ms_avg, launches)."""
    import torch

    from paper_2106_08950_amd import dilbm

    prm = dilbm.params_from_workload(wl, storage=storage, tile=tile, device=0,
                                     stream=stream.cuda_stream)
    s = dilbm.Solver(prm)
    s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    s.step(warmup)
    s.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    collide_ms, launches = s.kernel_timing()
    s.close()
    return wl.nodes * steps / dt / 1e6, dt, collide_ms / max(launches, 1), launches


def suspension3d_leg(steps, warmup, stream):
    """The three-dimensional path: 256^3 periodic D3Q19 nodes with 400 free spheres, FP32
    (19 x 4 bytes read + 19 x 4 written = 152 B per node update)."""
    import torch

    from paper_2106_08950_amd import dilbm3d, inputs3d

    w3 = inputs3d.suspension3d()
    s = dilbm3d.Solver3D(dilbm3d.params_from_workload(w3, device=0, stream=stream.cuda_stream))
    s.set_particles(w3.pos, w3.radius, w3.density, w3.vel, w3.omega, w3.fixed)
    s.step(warmup)
    s.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = s.kernel_timing()
    s.close()
    avg = ms / max(n, 1)
    a3 = 152 * w3.nodes / (avg * 1e-3) / 1e9
    return {"workload": w3.name, "value": round(w3.nodes * steps / dt / 1e6, 1),
            "unit": "MLUPS", "steps": steps, "ms_per_step": round(dt * 1e3 / steps, 4),
            "roofline": {"bound": "hbm", "achieved": round(a3, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(a3 / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic(COUNTERS3, KERNEL3_SRC),
                         "kernel": "k3_collide", "bytes_per_node": 152,
                         "avg_launch_ms": round(avg, 5), "launches": n}}


def batched_leg(stream, steps_per_solve=2000):
    """256-solve ensemble: one pool vs one plain solve after another."""
    import torch

    from paper_2106_08950_amd import dilbm, inputs

    wls = inputs.ensemble(nsteps=steps_per_solve)
    total = sum(w.nodes for w in wls) * steps_per_solve
    fp = sum(dilbm.footprint(dilbm.params_from_workload(w), w.nbodies) for w in wls)
    arena = torch.empty(int(fp * 1.05) + (64 << 20), dtype=torch.uint8, device="cuda")
    pool = dilbm.Pool(arena_bytes=arena.numel(), stream=stream.cuda_stream,
                      arena_ptr=arena.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [pool.submit(dilbm.params_from_workload(w), w.nsteps, w.pos, w.radius,
                           w.density, w.vel, w.omega, w.fixed) for w in wls]
    k, tile = pool.autotune(steps_per_trial=16)
    pool.run(steps_per_solve)
    pool.sync()
    dt_pool = time.perf_counter() - t0
    for t in tickets:
        assert pool.query(t) == (steps_per_solve, True)
    pool.close()
    del arena
    log(f"batched pool: {dt_pool:.2f} s, graph_steps={k}, tile={tile}")
    # the same solves, one plain solve after another
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w in wls:
        s = dilbm.Solver(dilbm.params_from_workload(w, stream=stream.cuda_stream))
        s.set_particles(w.pos, w.radius, w.density, w.vel, w.omega, w.fixed)
        s.step(steps_per_solve)
        s.close()
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    log(f"sequential plain solves: {dt_seq:.2f} s")
    return {"workload": f"ensemble of {len(wls)} solves x {steps_per_solve} steps",
            "node_updates": total,
            "pool_mlups": round(total / dt_pool / 1e6, 1),
            "sequential_mlups": round(total / dt_seq / 1e6, 1),
            "speedup": round(dt_seq / dt_pool, 2),
            "graph_steps": k, "tile": tile,
            "timing": "wall clock, admission + autotune + all steps (pool); create + "
                      "steps + destroy of each solve (sequential)"}


def served_leg(count=500):
    from paper_2106_08950_amd import inputs, serve

    reqs = inputs.request_stream(count=count)
    st = serve.serve(reqs, arena_bytes=200 << 30, chunk=64, graph_steps=32, tile=0,
                     realtime=True)
    log(f"served: {len(st.results)} done, makespan {st.makespan:.1f} s")
    return {"workload": f"request stream: {count} Poisson arrivals at 50/s",
            "completed": len(st.results), "rejected": st.rejected,
            "aggregate_mlups": round(st.mlups, 1),
            "p50_latency_s": round(st.percentile(50), 3),
            "p99_latency_s": round(st.percentile(99), 3),
            "makespan_s": round(st.makespan, 2),
            "arrival_span_s": round(reqs[-1][0], 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--legs", default="fp32,fp16,open_ends,suspension3d,batched,served")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--served-count", type=int, default=500)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to calibrate the HBM byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a slab decomposition along y is designed, not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))

    import torch

    from paper_2106_08950_amd import dilbm, inputs

    torch.cuda.init()
    stream = torch.cuda.Stream()
    wl = inputs.dense_suspension()

    log(f"fp32 {wl.name}: {args.steps} steps")
    mlups, dt, avg_ms, launches = single_solve(wl, dilbm.STORE_FP32, args.steps, args.warmup,
                                               args.tile, stream)
    achieved = 72 * wl.nodes / (avg_ms * 1e-3) / 1e9
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
                   "tau": wl.tau, "storage": "fp32", "tile": args.tile},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(), "kernel": "k_collide", "bytes_per_node": 72,
                     "avg_launch_ms": round(avg_ms, 5), "launches": launches},
    }
    cgbs = copy_reference(36 * wl.nodes)
    out["roofline"]["copy_GBs"] = round(cgbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / cgbs, 4)
    if "fp16" in legs:
        log("fp16")
        m16, dt16, avg16, n16 = single_solve(wl, dilbm.STORE_FP16, args.steps, args.warmup,
                                             args.tile, stream)
        a16 = 36 * wl.nodes / (avg16 * 1e-3) / 1e9
        out["fp16"] = {"value": round(m16, 1), "unit": "MLUPS",
                       "ms_per_step": round(dt16 * 1e3 / args.steps, 4),
                       "roofline": {"bound": "hbm", "achieved": round(a16, 1),
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(a16 / HBM_PEAK_GBS, 4), "bytes_per_node": 36,
                                    "traffic": measured_traffic(COUNTERS16),
                                    "avg_launch_ms": round(avg16, 5)}}
    if "open_ends" in legs:
        log("open ends")
        wo = inputs.inflow_array()
        mo, dto, avgo, no = single_solve(wo, dilbm.STORE_FP32, args.steps // 2, args.warmup,
                                         args.tile, stream)
        ao = 72 * wo.nodes / (avgo * 1e-3) / 1e9
        out["open_ends"] = {"workload": wo.name, "value": round(mo, 1), "unit": "MLUPS",
                            "ms_per_step": round(dto * 1e3 / (args.steps // 2), 4),
                            "roofline": {"bound": "hbm", "achieved": round(ao, 1),
                                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": round(ao / HBM_PEAK_GBS, 4),
                                         "bytes_per_node": 72, "avg_launch_ms": round(avgo, 5)}}
    if "suspension3d" in legs:
        log("suspension3d")
        out["suspension3d"] = suspension3d_leg(args.steps // 2, args.warmup, stream)
    if "batched" in legs:
        log("batched")
        out["batched"] = batched_leg(stream)
    if "served" in legs:
        log("served")
        out["served"] = served_leg(args.served_count)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = run_oracle_sample(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
