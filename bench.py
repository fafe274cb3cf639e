"""Benchmark of the DI-LBM time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--legs fp32,fp16,open_ends,suspension3d,suspension3d_q27,
                            suspension3d_fp16,open_ends3d,batched3d,batched,served]
                    [--no-cpu]

Headline workload (one step = the whole hot path over one solve): the dense suspension of
4096 x 4096 periodic nodes with 2000 free discs of radius 8 (seed 3), tau = 0.6, body
force 1e-6, FP32 shifted-population storage -- its 1.2 GB working set exceeds the 256 MB
Infinity Cache, so the populations stream from HBM every step.  Inputs are resident in
HBM before the timed region starts.

How each single-solve leg is measured:
1. set-up (create, bodies) on the host;
2. the copy bandwidth, the roofline's second denominator: device copies of the population
   volume back to back on the solve's stream;
3. a settle phase: untimed calls of K steps of the same solve for about 0.3 s.  After an
   idle spell the first ~60 steps (10-15 ms of streaming) run up to 10% slower while the
   chip's clocks settle (kernel traces show it; back-to-back copies before the steps
   shorten the transient but do not remove it), so a short timed region right after
   set-up would measure the transient rather than the step; calls of K steps also capture
   the K-step graph the timed runs replay;
4. W warm-up steps, then five timed runs of exactly K steps each (production path: HIP
   graph chunks), each bracketed by device synchronisations; `value` and `ms_per_step`
   come from the median run, and all five are reported;
5. a separate pass of max(K, 200) steps with HIP events around every collide launch on
   the solve's stream (direct launches): the roofline's per-launch average, with the
   minimum and the median.

Further legs, reported in the same JSON line:
* fp16: the same workload with FP16 storage (36 B per node update);
* open_ends: a 4096 x 2048 inflow channel (velocity inlet, zero-gradient outlet, 300
  fixed discs), FP32;
* suspension3d: the three-dimensional path, 256^3 D3Q19 nodes with 400 free spheres
  (seed 8), FP32 (152 B per node update);
* suspension3d_q27: the same on the D3Q27 lattice (216 B per node update);
* suspension3d_fp16: the D3Q19 suspension with FP16 storage (76 B per node update);
* open_ends3d: a 256^3 D3Q19 duct (diffuse walls in y and z) with a parabolic velocity
  inlet and a density outlet, past 200 fixed spheres, FP32;
* batched3d: 256 independent D3Q19 solves (sides 32-96, 1-3 spheres) advanced by one
  dilbm3d_batch_step, against the same solves stepped one after another;
* batched: the 256-solve ensemble (2000 steps each) advanced as one pool, against the
  same solves run one after another as plain solves;
* served: the 500-request Poisson stream (50 requests/s) through the continuous-batching
  loop, with p50/p99 completion latency.
Prints one JSON line.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, FP32 vs batched/FP16; p50/p99 latency of served solves"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2106_08950_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2106_08950_amd", "build.py")
# everything the collide kernels are compiled from (sources, headers, flags)
KERNEL_FILES = [os.path.join(CSRC, f) for f in
                ("kernels.hip", "kernels.h", "dilbm_internal.h", "device_common.h")] + [BUILD]
KERNEL3_FILES = [os.path.join(CSRC, f) for f in
                 ("kernels3d.hip", "kernels3d.h", "dilbm3d_internal.h", "device_common.h")] + [
                     BUILD]
COUNTERS = os.path.join(ROOT, "profiles", "k_collide_dense_suspension_4096_fp32_hbm_counters.txt")
COUNTERS16 = os.path.join(ROOT, "profiles", "k_collide_dense_suspension_4096_fp16_hbm_counters.txt")
COUNTERS_OPEN = os.path.join(ROOT, "profiles", "k_collide_inflow_4096x2048_fp32_hbm_counters.txt")
COUNTERS3 = os.path.join(ROOT, "profiles", "k3_collide_suspension3d_256_fp32_hbm_counters.txt")
COUNTERS3_27 = os.path.join(ROOT, "profiles",
                            "k3_collide_suspension3d_256_d3q27_fp32_hbm_counters.txt")
COUNTERS3_16 = os.path.join(ROOT, "profiles", "k3_collide_suspension3d_256_fp16_hbm_counters.txt")
COUNTERS3_OPEN = os.path.join(ROOT, "profiles", "k3_collide_inflow_duct3d_256_fp32_hbm_counters.txt")
TIMED_RUNS = 5


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(files=None):
    """Digest of every file the collide kernels are built from (the 2-D set by default)."""
    import hashlib

    h = hashlib.sha256()
    for path in files or KERNEL_FILES:
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(counters=None, files=None):
    """HBM bytes per collide launch from a committed rocprofv3 counter summary (default:
    the 2-D headline's), or None when a kernel source, header or the build flags have
    changed since the counters were taken."""
    try:
        with open(counters or COUNTERS) as f:
            kv = dict(ln.split(":", 1) for ln in f.read().splitlines() if ":" in ln)
    except OSError:
        return None
    if kv.get("kernel_source_sha256_16", "").strip() != kernel_source_hash(files):
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


def copy_bandwidth(stream, nbytes, seconds=0.2):
    """Back-to-back device copies of nbytes on `stream` for about `seconds`, with no host
    wait between them.  Returns the copy bandwidth (GB/s, nbytes read + nbytes written
    per copy) over the second half."""
    import torch

    n = max(nbytes // 4, 1)
    with torch.cuda.stream(stream):
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(8):
            y.copy_(x)
        b.record(stream)
        torch.cuda.synchronize()
        per = max(a.elapsed_time(b) / 8, 1e-3)  # ms per copy
        reps = max(16, int(seconds * 1e3 / per))
        for _ in range(reps // 2):
            y.copy_(x)
        a.record(stream)
        for _ in range(reps - reps // 2):
            y.copy_(x)
        b.record(stream)
        b.synchronize()
        gbs = 2 * n * 4 * (reps - reps // 2) / (a.elapsed_time(b) * 1e-3) / 1e9
        del x, y
    return gbs


def settle_steps(step, chunk, seconds=0.3):
    """Untimed calls of `chunk` steps of the solve for about `seconds` (see the module
    docstring); the calls are the timed runs' own length, so the timed runs replay a
    graph already captured."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        step(chunk)
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            break


def timed_runs(step, steps):
    """TIMED_RUNS runs of exactly `steps` steps, each between two device synchronisations;
    returns the wall seconds of each."""
    import torch

    out = []
    for _ in range(TIMED_RUNS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(steps)
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return out


def launch_pass(solver, steps):
    """Per-launch collide durations (ms) over `steps` directly launched, event-bracketed
    steps."""
    solver.set_kernel_timing(True)
    solver.step(steps)
    ms = list(solver.kernel_launch_times())
    solver.set_kernel_timing(False)
    return ms


def roofline(bytes_per_node, nodes, ms, traffic, kernel, copy_gbs=None):
    avg = sum(ms) / len(ms)
    achieved = bytes_per_node * nodes / (avg * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
         "bytes_per_node": bytes_per_node, "avg_launch_ms": round(avg, 5),
         "min_launch_ms": round(min(ms), 5), "median_launch_ms": round(statistics.median(ms), 5),
         "launches": len(ms), "timing": "HIP events around each collide launch on the "
                                       "solve's stream, separate pass after the timed runs"}
    if copy_gbs:
        r["copy_GBs"] = round(copy_gbs, 1)
        r["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return r


def single_solve(wl, storage, steps, warmup, tile, stream, bytes_per_node, traffic):
    """The measurement of one single-solve leg (see the module docstring)."""
    from paper_2106_08950_amd import dilbm

    prm = dilbm.params_from_workload(wl, storage=storage, tile=tile, device=0,
                                     stream=stream.cuda_stream)
    s = dilbm.Solver(prm)
    s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    copy_gbs = copy_bandwidth(stream, 9 * wl.nodes * (4 if storage == dilbm.STORE_FP32 else 2))
    settle_steps(s.step, steps)
    s.step(warmup)
    runs = timed_runs(s.step, steps)
    ms = launch_pass(s, max(steps, 200))
    s.close()
    dt = statistics.median(runs)
    return {"value": round(wl.nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt * 1e3 / steps, 4),
            "runs_ms_per_step": [round(r * 1e3 / steps, 4) for r in runs],
            "roofline": roofline(bytes_per_node, wl.nodes, ms, traffic, "k_collide", copy_gbs)}


def suspension3d_leg(steps, warmup, stream, q=19, storage=0, w3=None):
    """The three-dimensional path: 256^3 periodic nodes with 400 free spheres (or w3), on
    D3Q19 (19 x 4 bytes read + 19 x 4 written = 152 B per node update in FP32, 76 B in
    FP16) or D3Q27 (216 B in FP32)."""
    from paper_2106_08950_amd import dilbm3d, inputs3d

    es = 2 if storage == 1 else 4
    periodic = w3 is None
    w3 = inputs3d.suspension3d() if periodic else w3
    s = dilbm3d.Solver3D(dilbm3d.params_from_workload(w3, device=0, stream=stream.cuda_stream,
                                                      lattice=q, storage=storage))
    s.set_particles(w3.pos, w3.radius, w3.density, w3.vel, w3.omega, w3.fixed)
    copy_gbs = copy_bandwidth(stream, q * es * w3.nodes)
    settle_steps(s.step, steps)
    s.step(warmup)
    runs = timed_runs(s.step, steps)
    ms = launch_pass(s, max(steps, 100))
    s.close()
    dt = statistics.median(runs)
    counters = ({(19, 0): COUNTERS3, (27, 0): COUNTERS3_27, (19, 1): COUNTERS3_16}.get((q, storage))
                if periodic else (COUNTERS3_OPEN if (q, storage) == (19, 0) else None))
    return {"workload": w3.name, "lattice": f"D3Q{q}", "storage": "fp16" if storage else "fp32",
            "value": round(w3.nodes * steps / dt / 1e6, 1),
            "unit": "MLUPS", "steps": steps, "ms_per_step": round(dt * 1e3 / steps, 4),
            "runs_ms_per_step": [round(r * 1e3 / steps, 4) for r in runs],
            "roofline": roofline(2 * es * q, w3.nodes, ms,
                                 measured_traffic(counters, KERNEL3_FILES) if counters else None,
                                 "k3_collide", copy_gbs)}


def batched3d_leg(stream, steps=400):
    """The 3-D batch: 256 independent D3Q19 solves (inputs3d.ensemble3d) advanced together
    by dilbm3d_batch_step, against the same solves stepped one after another."""
    from paper_2106_08950_amd import dilbm3d, inputs3d

    wls = inputs3d.ensemble3d(nsteps=steps)
    nodes = sum(w.nodes for w in wls)

    def make():
        out = []
        for w in wls:
            s = dilbm3d.Solver3D(dilbm3d.params_from_workload(w, device=0,
                                                              stream=stream.cuda_stream))
            s.set_particles(w.pos, w.radius, w.density, w.vel, w.omega, w.fixed)
            out.append(s)
        return out

    members = make()
    batch = dilbm3d.Batch3D(members)
    batch.step(32)  # warm-up
    t0 = time.perf_counter()
    batch.step(steps)
    dt_batch = time.perf_counter() - t0
    batch.close()
    for s in members:
        s.close()
    solos = make()
    for s in solos:
        s.step(8)  # warm-up
    torch_sync(stream)
    t0 = time.perf_counter()
    for s in solos:
        s.step(steps)
    dt_seq = time.perf_counter() - t0
    for s in solos:
        s.close()
    mlups = nodes * steps / dt_batch / 1e6
    log(f"3-D batch: {dt_batch:.2f} s, one after another {dt_seq:.2f} s")
    return {"workload": f"ensemble of {len(wls)} D3Q19 solves x {steps} steps",
            "nodes": nodes, "batch_mlups": round(mlups, 1),
            "sequential_mlups": round(nodes * steps / dt_seq / 1e6, 1),
            "speedup": round(dt_seq / dt_batch, 2),
            "roofline": {"bound": "hbm", "bytes_per_node": 152,
                         "achieved": round(152 * mlups * 1e6 / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(152 * mlups * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
                         "timing": f"wall clock over {steps} steps of every member, whole "
                                   "step (collide + spheres)"},
            "timing": "batch: one dilbm3d_batch_step call after a 32-step warm-up; "
                      "sequential: dilbm3d_step of each solve in turn"}


def torch_sync(stream):
    stream.synchronize()


def batched_leg(stream, steps_per_solve=2000, window=256):
    """256-solve ensemble: one pool against one plain solve after another."""
    import torch

    from paper_2106_08950_amd import dilbm, inputs

    wls = inputs.ensemble(nsteps=steps_per_solve)
    nodes = sum(w.nodes for w in wls)
    total = nodes * steps_per_solve
    fp = sum(dilbm.footprint(dilbm.params_from_workload(w), w.nbodies) for w in wls)
    arena = torch.empty(int(fp * 1.05) + (64 << 20), dtype=torch.uint8, device="cuda")
    pool = dilbm.Pool(arena_bytes=arena.numel(), stream=stream.cuda_stream,
                      arena_ptr=arena.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [pool.submit(dilbm.params_from_workload(w), w.nsteps, w.pos, w.radius,
                           w.density, w.vel, w.omega, w.fixed) for w in wls]
    torch.cuda.synchronize()
    t_admit = time.perf_counter() - t0
    k, tile = pool.autotune(steps_per_trial=16)
    pool.sync()
    t_tune = time.perf_counter() - t0 - t_admit
    tuned = pool.query(tickets[0])[0]
    # steady state: a window of steps while every member is active
    pool.run(window)
    pool.sync()
    t1 = time.perf_counter()
    pool.run(window)
    pool.sync()
    dt_win = time.perf_counter() - t1
    pool.run(steps_per_solve)
    pool.sync()
    dt_pool = time.perf_counter() - t0
    for t in tickets:
        assert pool.query(t) == (steps_per_solve, True)
    pool.close()
    del arena
    steady = nodes * window / dt_win / 1e6
    log(f"batched pool: {dt_pool:.2f} s, graph_steps={k}, tile={tile}, autotune {tuned} steps")
    # the same solves as plain solves, one after another; each handle is created and its
    # graph captured (one untimed 32-step chunk) before the timed region
    solvers = []
    for w in wls:
        s = dilbm.Solver(dilbm.params_from_workload(w, stream=stream.cuda_stream))
        s.set_particles(w.pos, w.radius, w.density, w.vel, w.omega, w.fixed)
        s.step(32)
        solvers.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps_per_solve)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    for s in solvers:
        s.close()
    log(f"sequential plain solves: {dt_seq:.2f} s")
    seq = total / dt_seq / 1e6
    return {"workload": f"ensemble of {len(wls)} solves x {steps_per_solve} steps",
            "node_updates": total,
            "pool_mlups_steady": round(steady, 1),
            "pool_roofline": {"bound": "hbm", "bytes_per_node": 72,
                              "achieved": round(72 * steady * 1e6 / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(72 * steady * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
                              "timing": f"wall clock over {window} steps of every member "
                                        "after autotune, whole step (collide + bodies)"},
            "pool_mlups_wall": round(total / dt_pool / 1e6, 1),
            "sequential_mlups": round(seq, 1),
            "speedup_steady": round(steady / seq, 2),
            "speedup_wall": round(dt_seq / dt_pool, 2),
            "graph_steps": k, "tile": tile, "autotune_steps": tuned,
            "admission_s": round(t_admit, 3), "autotune_s": round(t_tune, 3),
            "timing": "pool_mlups_wall: admission + autotune + all steps; sequential: the "
                      "timed steps of each plain solve, handles created and graphs captured "
                      "beforehand"}


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, steps_all=4, steps_one=1, reps=3):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: `reps` runs
    of `steps_all` steps on all the threads OpenMP is given, then `reps` runs of
    `steps_one` steps on one thread; steady clock around the step loop (set-up excluded),
    median of the runs.  About 15-25 s on a 16-thread host share."""
    import oracle

    oracle.build_oracle(force=False)
    p = oracle.OracleParams(nx=wl.nx, ny=wl.ny, tau=wl.tau, rho0=wl.rho0, eps=wl.eps,
                            cutoff=wl.cutoff, G=tuple(wl.G), g=tuple(wl.g),
                            wall_mask=wl.wall_mask, wall_h=wl.wall_h, force_mode=wl.force_mode)
    s = oracle.OracleSolver(p)
    s.set_particles(wl.pos, wl.radius, wl.density, wl.vel, wl.omega, wl.fixed)
    threads = oracle.num_threads()

    def runs(n):
        out = []
        for _ in range(reps):
            t0 = time.perf_counter()
            s.step(n)
            out.append(time.perf_counter() - t0)
        return out

    s.step(1)  # warm
    t_all = runs(steps_all)
    oracle.set_num_threads(1)
    t_one = runs(steps_one)
    oracle.set_num_threads(threads)
    s.close()
    m_all = wl.nodes * steps_all / statistics.median(t_all) / 1e6
    m_one = wl.nodes * steps_one / statistics.median(t_one) / 1e6
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": round(m_all, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "one_thread": {"value": round(m_one, 3), "unit": "MLUPS", "cores": 1},
            "cpu_model": cpu_model(), "nproc": affinity,
            "sample": f"{wl.name}: FP64 oracle, median of {reps} runs of {steps_all} steps on "
                      f"{threads} OpenMP threads ({', '.join(f'{t:.2f}' for t in t_all)} s) "
                      f"and of {reps} runs of {steps_one} step on 1 thread "
                      f"({', '.join(f'{t:.2f}' for t in t_one)} s), after 1 warm-up step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--legs", default="fp32,fp16,open_ends,suspension3d,suspension3d_q27,"
                                      "suspension3d_fp16,open_ends3d,batched3d,batched,served")
    ap.add_argument("--no-cpu", action="store_true")
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

    log(f"fp32 {wl.name}: {TIMED_RUNS} x {args.steps} steps")
    r32 = single_solve(wl, dilbm.STORE_FP32, args.steps, args.warmup, args.tile, stream, 72,
                       measured_traffic())
    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "bodies": wl.nbodies,
                   "tau": wl.tau, "storage": "fp32", "tile": args.tile},
        "timed_runs": TIMED_RUNS,
        "runs_ms_per_step": r32["runs_ms_per_step"],
        "roofline": r32["roofline"],
    }
    if "fp16" in legs:
        log("fp16")
        out["fp16"] = single_solve(wl, dilbm.STORE_FP16, args.steps, args.warmup, args.tile,
                                   stream, 36, measured_traffic(COUNTERS16))
    if "open_ends" in legs:
        log("open ends")
        wo = inputs.inflow_array()
        r = single_solve(wo, dilbm.STORE_FP32, args.steps, args.warmup, args.tile, stream, 72,
                         measured_traffic(COUNTERS_OPEN))
        out["open_ends"] = {"workload": wo.name, **r}
    if "suspension3d" in legs:
        log("suspension3d")
        out["suspension3d"] = suspension3d_leg(max(args.steps // 2, 1), args.warmup, stream)
    if "suspension3d_q27" in legs:
        log("suspension3d D3Q27")
        out["suspension3d_q27"] = suspension3d_leg(max(args.steps // 2, 1), args.warmup,
                                                   stream, q=27)
    if "suspension3d_fp16" in legs:
        log("suspension3d FP16")
        out["suspension3d_fp16"] = suspension3d_leg(max(args.steps // 2, 1), args.warmup,
                                                    stream, q=19, storage=1)
    if "open_ends3d" in legs:
        log("open ends 3-D")
        from paper_2106_08950_amd import inputs3d

        out["open_ends3d"] = suspension3d_leg(max(args.steps // 2, 1), args.warmup, stream,
                                              w3=inputs3d.inflow_duct3d())
    if "batched3d" in legs:
        log("batched 3-D")
        out["batched3d"] = batched3d_leg(stream)
    if "batched" in legs:
        log("batched")
        out["batched"] = batched_leg(stream)
    if "served" in legs:
        log("served")
        out["served"] = served_leg(args.served_count)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
