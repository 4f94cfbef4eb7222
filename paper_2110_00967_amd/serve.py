"""Continuous-batching request loop for VP-LBM solves on one GPU.

Requests (a lattice description plus a number of steps) arrive over time.
The server:
  * admits a waiting request as soon as its device bytes
    (``vplbm_required_bytes``) fit in the HBM budget, keeping its lattice
    resident until it finishes;
  * advances resident lattices together, a chunk of steps at a time, with
    one batched launch per step (``vplbm_batch_step``); a request whose step
    count ends inside a chunk drops out of the launches at that point.  Which
    resident lattices run in a chunk is the policy: ``fair`` runs all of them;
    ``srpt`` runs those with the least remaining work (cells x steps) first,
    adding more until the chunk's lattices hold ``saturate_cells`` cells
    (enough to keep the GPU's memory system busy), while the others wait,
    resident, for a later chunk;
  * between chunks, retires finished requests (frees their memory, records the
    result) and admits newly arrived ones -- requests that arrive while
    others run join them at the next chunk boundary.
Every lattice computes exactly what it would alone (same kernels, same tiles,
same reduction order), so a request's result does not depend on the mix.

The engine is injectable so that the scheduling can be exercised without a
GPU; ``GpuEngine`` is the real one.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    case: Any                 # lattice description (workloads.Case-like)
    steps: int
    nbytes: int = 0
    handle: Any = None
    remaining: int = 0
    t_admit: Optional[float] = None
    t_finish: Optional[float] = None
    result: Any = None
    rejected: bool = False

    @property
    def cells(self):
        return self.case.nx * self.case.ny

    @property
    def latency(self):
        return None if self.t_finish is None else self.t_finish - self.arrival


class GpuEngine:
    """Lattices in torch-allocated HBM, stepped through the C ABI."""

    def __init__(self, precision="f32", streaming=0, tile=None):
        import torch

        from . import vplbm as V

        self.V, self.torch, self.precision = V, torch, precision
        self.streaming = int(streaming)  # STREAM_AB or STREAM_AA (half the population memory)
        self._batch = None
        self._batch_key = None
        self.tile = tile  # tile of the batched launches (None: the library's default)
        self.batches_created = 0

    def _params(self, case):
        # the parameters create() builds its lattice from
        return self.V.case_params(case, self.precision, hist_capacity=16, streaming=self.streaming)

    def nbytes(self, case):
        return self.V.required_bytes(self._params(case))

    def create(self, case):
        return self.V.Lattice.from_case(case, precision=self.precision, hist_capacity=16, streaming=self.streaming)

    def step(self, handles, nsteps):
        # one batch for the engine's lifetime: a new resident set only
        # replaces its lattices (vplbm_batch_set_lattices), so membership
        # changes cost no device allocation, stream or graph rebuild beyond
        # a new launch shape
        key = tuple(id(h) for h in handles)
        if self._batch is None:
            self._batch = self.V.Batch(handles)
            self.batches_created += 1
            if self.tile is not None:
                self._batch.set_tile(*self.tile)
        elif key != self._batch_key:
            self._batch.set_lattices(handles)
        self._batch_key = key
        self._batch.step(nsteps)

    def sync(self):
        self.torch.cuda.synchronize()

    def result(self, h):
        return {"me": h.forces_me().tolist(), "si": h.forces_si().tolist(), "body": h.body_state().tolist(),
                "steps": h.step_count}

    def release(self, h):
        if self._batch is not None and id(h) in (self._batch_key or ()):
            # the batch must not keep a destroyed lattice: the next step()
            # hands it the new resident set
            self._batch_key = None
        h.close()
        h._buf = None

    def close(self):
        if self._batch is not None:
            self._batch.close()
            self._batch, self._batch_key = None, None


class Server:
    """Continuous batching under an HBM budget (see the module docstring)."""

    def __init__(self, engine, budget_bytes: int, chunk: int = 1000, max_resident: int = 256,
                 clock: Optional[Callable[[], float]] = None, sleep: Optional[Callable[[float], None]] = None,
                 policy: str = "fair", saturate_cells: int = 4 << 20):
        if policy not in ("fair", "srpt"):
            raise ValueError(f"unknown policy {policy!r}")
        self.engine = engine
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.max_resident = int(max_resident)
        self.policy = policy
        self.saturate_cells = int(saturate_cells)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.events: List[tuple] = []   # (time, kind, rid) for inspection
        self.peak_bytes = 0             # most resident bytes at any time
        self.peak_resident = 0          # most resident requests at any time

    def _chunk_steps(self, resident: List[Request]) -> List[int]:
        """Steps each resident request advances in the next chunk (0 = waits)."""
        if self.policy == "fair":
            return [min(r.remaining, self.chunk) for r in resident]
        order = sorted(range(len(resident)),
                       key=lambda i: (resident[i].remaining * resident[i].cells, resident[i].arrival, resident[i].rid))
        n = [0] * len(resident)
        cells = 0
        for i in order:
            n[i] = min(resident[i].remaining, self.chunk)
            cells += resident[i].cells
            if cells >= self.saturate_cells:
                break
        return n

    def run(self, items, progress: Optional[Callable[[int, int, float], None]] = None) -> List[Request]:
        """items: iterable of (rid, arrival_s, case, steps). Returns the requests.
        progress(finished, total, t) is called after every request that finishes."""
        reqs = [Request(rid, float(t), case, int(n)) for rid, t, case, n in items]
        for r in reqs:
            r.nbytes = self.engine.nbytes(r.case)
            r.remaining = r.steps
        future = collections.deque(sorted(reqs, key=lambda r: (r.arrival, r.rid)))
        waiting: collections.deque = collections.deque()
        resident: List[Request] = []
        used = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0
        while future or waiting or resident:
            t = now()
            while future and future[0].arrival <= t:
                r = future.popleft()
                if r.nbytes > self.budget:
                    r.rejected = True
                    self.events.append((t, "reject", r.rid))
                    continue
                waiting.append(r)
            # admission in arrival order; a request that does not fit waits
            # for memory, and so do the ones behind it (no overtaking)
            while waiting and len(resident) < self.max_resident and used + waiting[0].nbytes <= self.budget:
                r = waiting.popleft()
                r.handle = self.engine.create(r.case)
                r.t_admit = now()
                used += r.nbytes
                resident.append(r)
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_resident = max(self.peak_resident, len(resident))
                self.events.append((r.t_admit, "admit", r.rid))
            if not resident:
                if future:
                    self.sleep(max(0.0, future[0].arrival - now()))
                continue
            n = self._chunk_steps(resident)
            self.engine.step([r.handle for r in resident], n)
            self.engine.sync()
            t = now()
            still = []
            for r, k in zip(resident, n):
                r.remaining -= k
                if r.remaining == 0:
                    r.t_finish = t
                    r.result = self.engine.result(r.handle)
                    self.engine.release(r.handle)
                    r.handle = None
                    used -= r.nbytes
                    self.events.append((t, "finish", r.rid))
                    if progress:
                        progress(sum(1 for e in self.events if e[1] == "finish"), len(reqs), t)
                else:
                    still.append(r)
            resident = still
        return reqs


def serial_run(engine, items, clock=None, sleep=None) -> List[Request]:
    """The plain form: one request at a time, in arrival order, each alone."""
    clock = clock or time.perf_counter
    sleep = sleep or time.sleep
    reqs = sorted((Request(rid, float(t), case, int(n)) for rid, t, case, n in items),
                  key=lambda r: (r.arrival, r.rid))
    t0 = clock()
    for r in reqs:
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        r.handle = engine.create(r.case)
        r.t_admit = clock() - t0
        engine.step([r.handle], [r.steps])
        engine.sync()
        r.t_finish = clock() - t0
        r.result = engine.result(r.handle)
        engine.release(r.handle)
        r.handle = None
    return reqs


def percentile(values, q):
    v = sorted(values)
    if not v:
        return math.nan
    k = (len(v) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def summarize(reqs: List[Request]) -> dict:
    done = [r for r in reqs if r.t_finish is not None]
    lat = [r.latency for r in done]
    span = max((r.t_finish for r in done), default=0.0) - min((r.arrival for r in done), default=0.0)
    work = sum(r.cells * r.steps for r in done)
    return {"requests": len(reqs), "completed": len(done), "rejected": sum(r.rejected for r in reqs),
            "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
            "mean_latency_s": sum(lat) / len(lat) if lat else math.nan,
            "makespan_s": span, "aggregate_MLUPS": work / span / 1e6 if span > 0 else math.nan}
