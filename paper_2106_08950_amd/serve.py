"""Continuous-batching request loop over a dilbm pool.

Requests arrive over time (each a full DI-LBM solve: lattice, bodies, step count).  The
loop keeps one pool on one GPU and, every iteration:

1. admits waiting requests in arrival order while their device footprint fits in the
   pool's free arena (a request that cannot fit now waits; one larger than the whole
   arena is rejected);
2. enqueues `chunk` steps for every admitted solve (one collide launch and one body launch
   per step for all of them, captured in a HIP graph) without waiting for the GPU;
3. collects solves whose last step has completed: copies their fields and bodies to the
   host, records the completion time, and releases their memory.

State stays on the device between chunks; requests that arrive while others run join the
next chunk, so their work overlaps on the GPU.  The device arena is a torch allocation:
PyTorch provides the memory and the stream, the library does the rest.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import dilbm


@dataclass
class Result:
    index: int
    arrival: float          # seconds since the stream started
    admitted: float
    finished: float
    nodes: int
    steps: int
    rho: np.ndarray = None
    ux: np.ndarray = None
    uy: np.ndarray = None
    pos: np.ndarray = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    results: list = field(default_factory=list)
    makespan: float = 0.0
    node_updates: float = 0.0
    rejected: int = 0

    @property
    def mlups(self) -> float:
        return self.node_updates / self.makespan / 1e6 if self.makespan > 0 else 0.0

    def percentile(self, q) -> float:
        lat = [r.latency for r in self.results]
        return float(np.percentile(lat, q)) if lat else float("nan")


def serve(requests, arena_bytes: int, chunk: int = 64, graph_steps: int = 32, tile: int = 0,
          keep_fields: bool = False, realtime: bool = True, device: int = 0,
          clock=time.perf_counter) -> ServeStats:
    """Run a stream of (arrival_time_s, inputs.Workload) requests to completion.

    With ``realtime`` a request is only visible once its arrival time has passed on the
    wall clock, and latency runs from that time.  Otherwise the stream is an offline
    batch: every request arrives at time zero and is admitted in list order.
    """
    import torch

    torch.cuda.init()
    dev = torch.device("cuda", device)
    arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    pool = dilbm.Pool(arena_bytes=int(arena_bytes), device=device, stream=stream.cuda_stream,
                      arena_ptr=arena.data_ptr())
    pool.set_launch(graph_steps, tile)
    stats = ServeStats()
    pending = sorted(((t if realtime else 0.0, i, wl) for i, (t, wl) in enumerate(requests)),
                     key=lambda r: (r[0], r[1]))
    running = {}   # ticket -> (index, arrival, admitted, workload)
    t0 = clock()
    nxt = 0
    try:
        while nxt < len(pending) or running:
            now = clock() - t0
            # 1. admission, in arrival order, by footprint
            while nxt < len(pending) and (not realtime or pending[nxt][0] <= now):
                t_arr, idx, wl = pending[nxt]
                prm = dilbm.params_from_workload(wl, device=device)
                try:
                    ticket = pool.submit(prm, wl.nsteps, wl.pos, wl.radius, wl.density,
                                         wl.vel, wl.omega, wl.fixed)
                except dilbm.DilbmError as e:
                    if e.status != dilbm.ENOMEM:
                        raise
                    stats.rejected += 1
                    nxt += 1
                    continue
                if ticket is None:
                    break  # no room now; keep arrival order
                running[ticket] = (idx, t_arr, clock() - t0, wl)
                nxt += 1
            # 2. enqueue a chunk for every admitted solve
            if running:
                pool.run(chunk)
            # 3. collect finished solves
            done = [t for t in running if pool.query(t)[1]]
            if not done and running and pool.stats()[1] == 0:
                # every admitted solve has all its steps enqueued: nothing more to launch
                # until the GPU finishes them or a request arrives
                due = pending[nxt][0] - (clock() - t0) if nxt < len(pending) else None
                if due is None:
                    pool.sync()
                elif due > 0.0:
                    time.sleep(min(due, 0.002))
                done = [t for t in running if pool.query(t)[1]]
            for t in done:
                idx, t_arr, t_adm, wl = running.pop(t)
                r = Result(index=idx, arrival=t_arr, admitted=t_adm, finished=0.0,
                           nodes=wl.nodes, steps=wl.nsteps)
                if keep_fields:
                    r.rho, r.ux, r.uy = pool.get_fields(t)
                    r.pos = pool.get_particles(t)[0]
                else:
                    r.pos = pool.get_particles(t)[0]
                r.finished = clock() - t0
                pool.release(t)
                stats.results.append(r)
                stats.node_updates += wl.nodes * wl.nsteps
            if not running and nxt < len(pending) and realtime:
                wait = pending[nxt][0] - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
        pool.sync()
        stats.makespan = clock() - t0
    finally:
        pool.close()
        del arena
    stats.results.sort(key=lambda r: r.index)
    return stats
