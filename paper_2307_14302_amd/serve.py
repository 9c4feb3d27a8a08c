"""Continuous-batching request loop for flood scenarios (argument marshalling
and scheduling only; every step runs in libdgswe.so).

Requests arrive over time.  Each names a mesh of a pool that is uploaded
once and shared (``dgswe_share_mesh``), its own initial state and forcing,
and a step count.  Between chunks of batch steps the loop admits requests
that have arrived, in arrival order, while their device footprint fits the
HBM budget (``dgswe_batch_add`` refuses the rest), and retires the ones that
finished: their state is read to the host, which ends their latency.
Requests admitted while others run share every later launch with them
(``dgswe_batch_step``), so the device is never drained between requests.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _native as N
from .solver import Batch, Solver


@dataclass
class Request:
    id: int
    arrival: float                     # seconds after the loop starts
    mesh: object                       # key of a registered mesh
    n_steps: int
    initial: tuple                     # (zeta, qx, qy) nodal arrays
    rain: Dict[str, object]
    tides: Dict[int, tuple] = field(default_factory=dict)
    rivers: Dict[int, tuple] = field(default_factory=dict)
    # filled by the loop
    admitted: float = float("nan")
    done: float = float("nan")
    result: Optional[np.ndarray] = None
    mass: Optional[dict] = None
    error: Optional[str] = None        # set when the run latched a non-finite volume or step
    n_tri: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """One batch on one stream; ``params`` are shared by every request."""

    def __init__(self, params: Dict[str, object], budget_bytes: int, chunk_steps: int = 20,
                 keep_results: bool = True, result_layout: str = "vertex"):
        self.params = dict(params)
        self.budget = int(budget_bytes)
        self.chunk = int(chunk_steps)
        self.keep = keep_results
        self.layout = result_layout
        self.batch = Batch(self.params, budget_bytes=self.budget)
        self.meshes: Dict[object, Solver] = {}

    def register_mesh(self, key, xy, hb, fric, tri, bedges=None, btype=None, bslot=None):
        """Upload a pool mesh once; requests on it share its device arrays."""
        s = Solver(self.params)
        s.upload_mesh(xy, hb, fric, tri, bedges, btype, bslot)
        self.meshes[key] = s
        return s

    def _start(self, r: Request) -> Solver:
        s = Solver(self.params)
        s.share_mesh(self.meshes[r.mesh])
        for slot, (mean, rows) in r.tides.items():
            s.set_tide(slot, mean, rows)
        for slot, (t, q) in r.rivers.items():
            s.set_river(slot, t, q)
        s.set_rain(r.rain)
        s.set_initial_nodal(*r.initial)
        return s

    def run(self, requests: List[Request], clock: Callable[[], float] = time.perf_counter) -> List[Request]:
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        active: Dict[int, tuple] = {}
        finished: List[Request] = []
        t0 = clock()
        while pending or active:
            now = clock() - t0
            # admission in arrival order while the footprint fits
            while pending and pending[0].arrival <= now:
                r = pending[0]
                need = Solver.footprint_of(self.params, self.meshes[r.mesh])
                used = self.batch.info()[1]
                if active and used + need > self.budget:
                    break
                s = self._start(r)
                try:
                    slot = self.batch.add(s, r.n_steps)
                except N.DgsweError as e:
                    s.close()
                    if e.code == N.DGSWE_EBUDGET and active:
                        break
                    raise
                r.admitted = clock() - t0
                r.n_tri = s.n_tri
                active[slot] = (r, s)
                pending.popleft()
            if not active:
                # idle until the next arrival
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            self.batch.step(self.chunk)
            for slot in self.batch.poll():
                r, s = active.pop(slot)
                self.batch.retire(slot)
                try:
                    r.mass = s.mass()
                    res = s.state(self.layout)
                    if self.keep:
                        r.result = res
                except N.DgsweError as e:        # this request failed; the others go on
                    r.error = str(e)
                r.done = clock() - t0
                s.close()
                finished.append(r)
        return finished

    def close(self):
        self.batch.close()
        for s in self.meshes.values():
            s.close()
        self.meshes.clear()


def latency_summary(done: List[Request]) -> Dict[str, float]:
    """p50/p99/mean of the arrival -> result latency, split into the queue
    delay (arrival -> admission into the batch) and the service time
    (admission -> result on the host)."""
    lat = np.array([r.latency for r in done])
    queue = np.array([r.admitted - r.arrival for r in done])
    service = np.array([r.done - r.admitted for r in done])

    def pct(a, q):
        return float(np.percentile(a, q)) if a.size else None

    return {"n": int(lat.size), "failed": sum(1 for r in done if r.error),
            "p50_s": pct(lat, 50), "p99_s": pct(lat, 99), "mean_s": float(lat.mean()) if lat.size else None,
            "queue_p50_s": pct(queue, 50), "queue_p99_s": pct(queue, 99),
            "service_p50_s": pct(service, 50), "service_p99_s": pct(service, 99)}
