"""Request loop (continuous batching under an HBM budget).

CPU tests drive the scheduler with a counting engine and a simulated clock
(time advances with the work done), and check the admission invariants and
the latency bookkeeping.  The GPU test runs a small mixed trace through the
real engine and checks every request's result against the same request run
alone (bitwise)."""
import math
import types

import numpy as np
import pytest

import workloads as W
from paper_2110_00967_amd.serve import Server, percentile, serial_run, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class CountingEngine:
    """Stands in for the GPU: bytes ~ cells, time ~ cell updates."""

    def __init__(self, clock, rate=1e6):
        self.clock, self.rate = clock, rate
        self.live = {}
        self.steps = {}
        self.peak = 0
        self.bytes_live = 0
        self.launches = []
        self.active = []

    def nbytes(self, case):
        return case.nx * case.ny * 100

    def create(self, case):
        h = types.SimpleNamespace(case=case, id=len(self.steps))
        self.steps[h.id] = 0
        self.live[h.id] = self.nbytes(case)
        self.bytes_live += self.nbytes(case)
        self.peak = max(self.peak, self.bytes_live)
        return h

    def step(self, handles, nsteps):
        self.launches.append(len(handles))
        self.active.append(sum(1 for n in nsteps if n))
        work = 0
        for h, n in zip(handles, nsteps):
            self.steps[h.id] += n
            work += n * h.case.nx * h.case.ny
        self.clock.t += work / self.rate

    def sync(self):
        pass

    def result(self, h):
        return {"steps": self.steps[h.id]}

    def release(self, h):
        self.bytes_live -= self.live.pop(h.id)


def box(nx, ny):
    return types.SimpleNamespace(nx=nx, ny=ny)


def items_from(spec):
    return [(i, t, box(nx, ny), n) for i, (t, nx, ny, n) in enumerate(spec)]


def test_budget_fifo_and_completion():
    clk = Clock()
    eng = CountingEngine(clk)
    rng = np.random.default_rng(0)
    spec = [(float(t), int(nx), int(ny), int(n)) for t, nx, ny, n in
            zip(np.cumsum(rng.exponential(0.05, 60)), rng.choice([16, 32, 64], 60), rng.choice([16, 32], 60),
                rng.integers(50, 2000, 60))]
    budget = 64 * 32 * 100 * 3  # room for about three of the largest
    srv = Server(eng, budget, chunk=200, clock=clk, sleep=clk.sleep)
    reqs = srv.run(items_from(spec))
    assert eng.peak <= budget
    assert all(r.t_finish is not None and not r.rejected for r in reqs)
    assert all(r.result["steps"] == r.steps for r in reqs)
    assert all(r.arrival <= r.t_admit <= r.t_finish for r in reqs)
    admits = [rid for _, kind, rid in srv.events if kind == "admit"]
    order = [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert admits == order  # first come, first admitted
    assert max(eng.launches) >= 2  # several requests shared launches
    s = summarize(reqs)
    assert s["completed"] == 60 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_late_arrival_joins_running_batch():
    clk = Clock()
    eng = CountingEngine(clk, rate=1e4)
    # a long request, then a short one arriving while it runs
    spec = [(0.0, 32, 32, 10000), (1.0, 16, 16, 300)]
    srv = Server(eng, 10 ** 9, chunk=500, clock=clk, sleep=clk.sleep)
    r0, r1 = srv.run(items_from(spec))
    assert r1.t_admit < r0.t_finish  # admitted before the first one is done
    assert r1.t_finish < r0.t_finish
    assert r1.t_admit - r1.arrival <= 500 * 32 * 32 / 1e4 + 1e-9  # waited at most one chunk


def test_oversized_request_is_rejected_and_others_run():
    clk = Clock()
    eng = CountingEngine(clk)
    spec = [(0.0, 16, 16, 100), (0.0, 4096, 4096, 10), (0.1, 16, 16, 100)]
    reqs = Server(eng, 16 * 16 * 100 * 4, chunk=50, clock=clk, sleep=clk.sleep).run(items_from(spec))
    assert reqs[1].rejected and reqs[1].t_finish is None
    assert reqs[0].t_finish is not None and reqs[2].t_finish is not None


def test_idle_server_waits_for_arrivals():
    clk = Clock()
    eng = CountingEngine(clk)
    reqs = Server(eng, 10 ** 9, chunk=100, clock=clk, sleep=clk.sleep).run(items_from([(5.0, 8, 8, 10)]))
    assert reqs[0].t_admit >= 5.0


def test_serial_run_one_at_a_time():
    clk = Clock()
    eng = CountingEngine(clk)
    reqs = serial_run(eng, items_from([(0.0, 16, 16, 100), (0.0, 16, 16, 100)]), clock=clk, sleep=clk.sleep)
    assert reqs[1].t_admit >= reqs[0].t_finish
    assert eng.launches == [1, 1]


def test_srpt_short_request_overtakes_and_everything_finishes():
    # a long request, then short ones arriving while it runs: under srpt the
    # short ones run alone (each fills the saturation threshold) and finish
    # sooner than under fair sharing; the long one still finishes and every
    # request gets exactly its steps
    spec = [(0.0, 64, 64, 20000), (1.0, 16, 16, 300), (1.5, 16, 16, 300), (2.0, 32, 32, 500)]
    out = {}
    for policy in ("fair", "srpt"):
        clk = Clock()
        eng = CountingEngine(clk, rate=1e5)
        srv = Server(eng, 10 ** 9, chunk=100, clock=clk, sleep=clk.sleep, policy=policy, saturate_cells=16 * 16)
        reqs = srv.run(items_from(spec))
        assert all(r.result["steps"] == r.steps for r in reqs)
        out[policy] = (reqs, eng)
    fair, srpt = out["fair"][0], out["srpt"][0]
    for k in (1, 2, 3):
        assert srpt[k].latency < fair[k].latency
    assert srpt[0].t_finish is not None
    # the same total work: the last request finishes at the same time
    assert math.isclose(max(r.t_finish for r in srpt), max(r.t_finish for r in fair), rel_tol=1e-9)
    # srpt ran one request per chunk here (each one reaches the threshold)
    assert max(out["srpt"][1].active) == 1 and max(out["fair"][1].active) >= 2


def test_srpt_fills_the_saturation_threshold():
    clk = Clock()
    eng = CountingEngine(clk)
    spec = [(0.0, 16, 16, 1000 + 10 * i) for i in range(8)]
    srv = Server(eng, 10 ** 9, chunk=100, clock=clk, sleep=clk.sleep, policy="srpt", saturate_cells=3 * 256)
    reqs = srv.run(items_from(spec))
    assert all(r.result["steps"] == r.steps for r in reqs)
    assert max(eng.active) == 3  # three 16 x 16 lattices reach 768 cells
    # least remaining work first: finishing order follows the step counts
    order = sorted(reqs, key=lambda r: r.t_finish)
    assert [r.rid for r in order] == list(range(8))
    with pytest.raises(ValueError):
        Server(eng, 1, policy="lifo")


def test_percentile():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    assert percentile([5], 99) == 5
    assert math.isnan(percentile([], 50))


@pytest.mark.gpu
@pytest.mark.parametrize("streaming", [0, 1])
def test_gpu_mix_equals_alone(streaming):
    from gpu_cases import say
    from paper_2110_00967_amd import vplbm as V
    from paper_2110_00967_amd.serve import GpuEngine
    reqs = W.serving_trace(nreq=8, seed=3, rate=50.0, grids=((64, 64), (128, 64), (96, 96)),
                           steps_range=(60, 400))
    items = W.serving_items(reqs)
    say("serve 8 mixed requests (airfoil + sedimentation), fp32, storage", "AA" if streaming else "AB")
    eng = GpuEngine("f32", streaming=streaming)
    budget = 3 * eng.nbytes(items[0][2])
    out = Server(eng, budget, chunk=64).run(items)
    assert all(r.t_finish is not None for r in out)
    for r, (_, _, case, n) in zip(sorted(out, key=lambda r: r.rid), sorted(items, key=lambda i: i[0])):
        g = V.Lattice.from_case(case, precision="f32", hist_capacity=16, streaming=streaming)
        g.step(n)
        alone = {"me": g.forces_me().tolist(), "si": g.forces_si().tolist(), "body": g.body_state().tolist()}
        assert r.result["me"] == alone["me"] and r.result["si"] == alone["si"], r.rid
        assert r.result["body"] == alone["body"], r.rid
        g.close()
    s = summarize(out)
    say(f"served: p50 {s['p50_latency_s'] * 1e3:.1f} ms, p99 {s['p99_latency_s'] * 1e3:.1f} ms")
    # one batch served every resident set (membership changes replace its lattices)
    assert eng.batches_created == 1
    eng.close()
