"""The continuous-batching request loop: requests that arrive while others run are
admitted as memory frees up, and every result equals the same solve run alone (FP32
round-off only) and the FP64 oracle (stated tolerance)."""
import numpy as np
import pytest

from paper_2106_08950_amd import inputs, serve
from helpers import gpu_solver, log_case, oracle_solver, velocity_rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def _stream(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(count):
        t += float(rng.exponential(0.01))
        side = int(rng.integers(40, 200))
        nd = int(rng.integers(0, 6))
        pos, rad = inputs.place_discs(rng, side, side, nd, lambda r: r.uniform(3.0, 7.0))
        wl = inputs.Workload(name=f"req{k}", nx=side, ny=side,
                             tau=float(rng.uniform(0.55, 1.5)),
                             nsteps=int(rng.integers(50, 400)), eps=2.0,
                             G=(float(rng.uniform(1e-7, 1e-5)), 0.0),
                             **inputs._bodies(pos, rad, np.full(len(rad), 1.2)))
        out.append((t, wl))
    return out


def test_served_results_equal_alone_and_oracle():
    reqs = _stream(17, 24)
    log_case("serve 24 requests")
    # a small arena forces waiting for memory: about a third of the requests fit at once
    from paper_2106_08950_amd import dilbm

    fps = [dilbm.footprint(dilbm.params_from_workload(wl), wl.nbodies) for _, wl in reqs]
    arena = int(sum(fps) / 3) + (8 << 20)
    st = serve.serve(reqs, arena_bytes=arena, chunk=16, graph_steps=8, tile=0,
                     keep_fields=True, realtime=False)
    assert len(st.results) == len(reqs) and st.rejected == 0
    # offline batch: everything arrives at t = 0 and completes after its admission
    assert all(r.arrival == 0.0 and r.finished >= r.admitted >= 0.0 for r in st.results)
    for r in st.results:
        wl = reqs[r.index][1]
        g = gpu_solver(wl)
        g.step(wl.nsteps)
        _, ux, uy = g.get_fields()
        assert velocity_rel_l2(r.ux, r.uy, ux, uy) < 1e-6, wl.name
        if wl.nbodies:
            x, _, _ = g.get_particles()
            assert np.abs(r.pos - x).max() < 1e-7
        g.close()
    for r in st.results[::6]:
        wl = reqs[r.index][1]
        o = oracle_solver(wl)
        o.step(wl.nsteps)
        _, uxo, uyo = o.get_fields()
        assert velocity_rel_l2(r.ux, r.uy, uxo, uyo) < 1e-5, wl.name
    assert st.mlups > 0 and st.percentile(99) >= st.percentile(50)


def test_realtime_arrivals_while_others_run():
    """Requests that arrive on the wall clock while earlier ones run: each is admitted no
    earlier than its arrival time, some are admitted while others are still running, and
    every result equals the same solve run alone.  These solves run 1500-3000 steps, up to
    eight times the batch test's: the order-of-summation differences between the pooled and
    the lone run (body sums by atomics) grow with the step count, so positions get 1e-6
    (the batch test's 1e-7 scaled by the steps)."""
    rng = np.random.default_rng(23)
    reqs = []
    t = 0.0
    for k in range(16):
        t += float(rng.exponential(0.004))
        side = int(rng.integers(64, 160))
        pos, rad = inputs.place_discs(rng, side, side, int(rng.integers(0, 5)),
                                      lambda r: r.uniform(3.0, 6.0))
        reqs.append((t, inputs.Workload(name=f"rt{k}", nx=side, ny=side,
                                        tau=float(rng.uniform(0.6, 1.2)),
                                        nsteps=int(rng.integers(1500, 3000)), eps=2.0,
                                        G=(float(rng.uniform(1e-7, 5e-6)), 0.0),
                                        **inputs._bodies(pos, rad, np.full(len(rad), 1.2)))))
    log_case("serve 16 requests in real time")
    from paper_2106_08950_amd import dilbm

    fps = [dilbm.footprint(dilbm.params_from_workload(wl), wl.nbodies) for _, wl in reqs]
    arena = int(sum(fps) / 2) + (8 << 20)
    st = serve.serve(reqs, arena_bytes=arena, chunk=16, graph_steps=8, tile=0,
                     keep_fields=True, realtime=True)
    assert len(st.results) == len(reqs) and st.rejected == 0
    res = st.results
    for r in res:
        assert r.arrival == reqs[r.index][0]
        assert r.finished >= r.admitted >= r.arrival
    overlap = sum(any(a.admitted < b.admitted < a.finished for a in res if a is not b)
                  for b in res)
    print(f"realtime serve: {overlap} of {len(res)} admitted while another ran; "
          f"p50 {st.percentile(50):.3f} s, p99 {st.percentile(99):.3f} s")
    assert overlap > 0
    for r in res:
        wl = reqs[r.index][1]
        g = gpu_solver(wl)
        g.step(wl.nsteps)
        _, ux, uy = g.get_fields()
        assert velocity_rel_l2(r.ux, r.uy, ux, uy) < 1e-6, wl.name
        if wl.nbodies:
            x, _, _ = g.get_particles()
            assert np.abs(r.pos - x).max() < 1e-6
        g.close()
