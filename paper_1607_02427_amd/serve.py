"""Serving loop: replica simulations submitted over time, run with
continuous batching on one device.

Requests (systems with an `arrival` time in seconds and a step count
`steps`) wait in a FIFO queue until the device has room for them: a request
is admitted when its device footprint (dem_footprint_bytes plus its state
and outputs) fits in what is left of the memory budget and the batch of its
dimension has a free run of particle slots.  The budget is enforced twice:
here across both dimensions' batches, and by each batch itself
(dem_batch_add returns DEM_E_OOM over the budget it was created with); a
request that waits on memory is marked so in its record.  Admitted requests join a
replica batch (one per dimension) whose every dem_step advances all live
replicas at once; each replica carries its own step budget, so it stops
exactly at its requested step count, and it is retired (its state copied
out if asked, its slots freed) at the next poll.  The loop steps the
batches in chunks of `chunk` steps and polls between chunks, which is when
arrivals are admitted and finished requests retired: requests that arrive
while others are on the device join them without waiting for them.  The
two dimensions' batches run on streams of their own, so a chunk's 2D and
3D steps overlap on the device.  Each
batch retunes its pair-kernel shape whenever its live particle count has
doubled since the last tuning (the shape never changes results).

All arithmetic runs in libdem's kernels; this module only schedules calls.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, Dict, List, Optional

import numpy as np

from . import dem

STATE_BYTES_PER_PARTICLE = 16 * 8 + 4 * 4  # state and outputs the batch keeps per particle (FP64, int32)


@dataclasses.dataclass
class Record:
    index: int
    n: int
    steps: int
    dim: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    result: Optional[tuple] = None
    waited_on_memory: bool = False

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def request_bytes(system, precision: str) -> int:
    """Device bytes a request occupies while it runs."""
    n64 = (system.n + 63) // 64 * 64
    return dem.footprint_bytes(system, precision) + STATE_BYTES_PER_PARTICLE * n64


class Server:
    def __init__(self, budget_bytes: int, precision: str = "fp32", max_replicas: int = 256,
                 max_particles: Dict[int, int] = None, chunk: int = 50, keep_results: bool = False,
                 clock: Callable[[], float] = time.perf_counter):
        self.budget = int(budget_bytes)
        self.precision = precision
        self.max_replicas = max_replicas
        self.max_particles = max_particles or {2: 1 << 20, 3: 1 << 21}
        self.chunk = int(chunk)
        self.keep_results = keep_results
        self.clock = clock
        self.batches: Dict[int, dem.DemBatch] = {}
        self.tuned_at: Dict[int, int] = {}  # live particles of each batch when its pair shape was last tuned
        self.used = 0
        self.peak_used = 0

    def _batch(self, dim: int) -> dem.DemBatch:
        if dim not in self.batches:
            import torch
            # each dimension's batch on a stream of its own (default priority),
            # so the 2D and 3D steps of a chunk run side by side on the device
            self.batches[dim] = dem.DemBatch(dim, self.precision, max_replicas=self.max_replicas,
                                             max_particles=self.max_particles[dim], budget_bytes=self.budget,
                                             stream=torch.cuda.Stream())
        return self.batches[dim]

    def run(self, systems: List, log: Optional[Callable[[str], None]] = None) -> List[Record]:
        """Serves `systems` (each with `arrival` and `steps`) and returns one
        record per request with its admission and completion times, measured
        on this host's clock from the start of the call."""
        order = sorted(range(len(systems)), key=lambda k: systems[k].arrival)
        recs = [Record(k, s.n, int(s.steps), s.dim, float(s.arrival)) for k, s in enumerate(systems)]
        pending = deque(order)
        queue: deque = deque()
        live: Dict[tuple, int] = {}  # (dim, replica id) -> request index
        cost: Dict[int, int] = {}
        t0 = self.clock()
        while pending or queue or live:
            now = self.clock() - t0
            while pending and systems[pending[0]].arrival <= now:
                queue.append(pending.popleft())
            # admission, first come first served, skipping what does not fit yet
            for k in list(queue):
                s = systems[k]
                c = request_bytes(s, self.precision)
                if self.used + c > self.budget:
                    recs[k].waited_on_memory = True
                    continue
                try:
                    rid = self._batch(s.dim).add(s, steps=int(s.steps))
                except dem.DemError as e:
                    if e.status == 3:  # over the batch's budget, or no free slots of the right size yet
                        continue
                    raise
                queue.remove(k)
                live[(s.dim, rid)] = k
                cost[k] = c
                self.used += c
                self.peak_used = max(self.peak_used, self.used)
                recs[k].admitted = self.clock() - t0
            if not live:
                if pending:  # idle until the next arrival
                    wait = systems[pending[0]].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(wait)
                    continue
                if queue:
                    raise RuntimeError("a queued request can never be admitted (budget or slots too small)")
                break
            for dim, b in self.batches.items():
                n_live = sum(systems[k].n for (d, _), k in live.items() if d == dim)
                if n_live >= 2 * self.tuned_at.get(dim, 0) and n_live > 0:
                    # the pair-kernel shape follows the batch as it grows
                    b.tune_pairs(2)
                    self.tuned_at[dim] = n_live
                if n_live > 0:
                    b.step(self.chunk)
            for dim, b in self.batches.items():
                mine = [rid for d, rid in live if d == dim]
                if not mine:
                    continue
                left, _ = b.progress(max(mine) + 1)
                t = self.clock() - t0
                for rid in mine:
                    if left[rid] == 0:
                        k = live.pop((dim, rid))
                        if self.keep_results:
                            recs[k].result = b.read(rid)
                        b.remove(rid)
                        self.used -= cost.pop(k)
                        recs[k].finished = t
                        if log:
                            log(f"[serve] request {k} n={systems[k].n} steps={systems[k].steps} "
                                f"latency {recs[k].latency:.3f} s")
        return recs

    def close(self):
        for b in self.batches.values():
            b.close()
        self.batches = {}


def summarize(recs: List[Record]) -> dict:
    lat = np.array([r.latency for r in recs])
    work = sum(r.n * r.steps for r in recs)
    makespan = max(r.finished for r in recs) - min(r.arrival for r in recs)
    return dict(requests=len(recs), p50_latency_s=float(np.percentile(lat, 50)),
                p99_latency_s=float(np.percentile(lat, 99)), mean_latency_s=float(lat.mean()),
                makespan_s=float(makespan), particle_steps=int(work), value=work / makespan,
                waited_on_memory=int(sum(r.waited_on_memory for r in recs)))


def run_sequential(systems: List, precision: str = "fp64", clock: Callable[[], float] = time.perf_counter,
                   log: Optional[Callable[[str], None]] = None) -> List[Record]:
    """The same requests one at a time in arrival order, each as a single
    system (dem_create_system) on the given path."""
    order = sorted(range(len(systems)), key=lambda k: systems[k].arrival)
    recs = [Record(k, s.n, int(s.steps), s.dim, float(s.arrival)) for k, s in enumerate(systems)]
    t0 = clock()
    for k in order:
        s = systems[k]
        wait = s.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        recs[k].admitted = clock() - t0
        with dem.DemSystem(s, precision) as g:
            g.step(int(s.steps))
            g.sync()
        recs[k].finished = clock() - t0
        if log:
            log(f"[sequential] request {k} n={s.n} steps={s.steps} latency {recs[k].latency:.3f} s")
    return recs
