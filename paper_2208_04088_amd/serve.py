"""Serving loop: continuous batching of plate solves on one GPU.

Requests arrive over time, each a plate and a number of steps.  A waiting
request is admitted into the resident batch (slbm_batch_add) as soon as its
device footprint fits the HBM budget, first come first served.  Every
resident plate is advanced together, one launch per step for all of them,
`chunk` steps per round (each plate by at most its remaining steps).  After
each round the finished plates are read back, removed (their memory is freed
at once) and the queue is admitted again.  All state stays on the device
between rounds.

`run_one_at_a_time` serves the same requests with one plate on the device at
a time and plain per-plate launches, for comparison.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Iterable, List, Optional

import numpy as np

from . import slbm


@dataclasses.dataclass
class Request:
    arrival: float           # seconds after the start of the run
    plate: object            # slbm_workloads.geometry.Plate
    steps: int


@dataclasses.dataclass
class Result:
    index: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    sites: int
    diverged: bool
    rejected: bool = False
    u: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def wait(self) -> float:
        return self.admitted - self.arrival


def _readout(solver, keep):
    diverged = False
    try:
        solver.sync()
    except slbm.SlbmError as e:
        if e.code != -4:
            raise
        diverged = True
    u = solver.displacement()            # the result a client receives
    return diverged, (u if keep else None)


class Server:
    """Continuous batching under an HBM budget (bytes)."""

    def __init__(self, budget_bytes: int, precision: str = "fp32", chunk: int = 64, device: int = 0,
                 stream=None, launch=None):
        self.batch = slbm.Batch(budget_bytes, device=device, stream=stream)
        self.precision = precision
        self.chunk = int(chunk)
        self.peak_bytes = 0
        self.peak_resident = 0
        if launch is not None:
            self.batch.set_launch(*launch)

    def close(self):
        self.batch.close()

    def run(self, requests: Iterable[Request], keep_results: bool = False,
            clock=time.perf_counter, sleep=time.sleep) -> List[Result]:
        reqs = list(requests)
        order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
        pending = collections.deque(order)
        waiting = collections.deque()
        resident = {}                     # slot -> (request index, admitted time)
        results: List[Optional[Result]] = [None] * len(reqs)
        t0 = clock()
        while pending or waiting or resident:
            now = clock() - t0
            while pending and reqs[pending[0]].arrival <= now:
                waiting.append(pending.popleft())
            # admission, first come first served, while the head fits
            while waiting:
                i = waiting[0]
                r = reqs[i]
                try:
                    slot = self.batch.add(r.plate, r.steps, self.precision)
                except slbm.SlbmError as e:
                    if e.code != -6:
                        raise
                    if not resident:
                        # larger than the whole budget: it can never run
                        waiting.popleft()
                        t = clock() - t0
                        results[i] = Result(i, r.arrival, t, t, r.steps, r.plate.n_material, False, True)
                        continue
                    break
                waiting.popleft()
                resident[slot] = (i, clock() - t0)
            used = self.batch.bytes()[0]
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_resident = max(self.peak_resident, len(resident))
            if not resident:
                if pending:
                    sleep(max(0.0, reqs[pending[0]].arrival - (clock() - t0)))
                continue
            self.batch.step(self.chunk)
            self.batch.sync()
            for slot in self.batch.poll():
                i, adm = resident.pop(slot)
                r = reqs[i]
                diverged, u = _readout(self.batch.solver(slot), keep_results)
                self.batch.remove(slot)
                results[i] = Result(i, r.arrival, adm, clock() - t0, r.steps, r.plate.n_material,
                                    diverged, False, u)
        return results


def run_one_at_a_time(requests: Iterable[Request], precision: str = "fp32", device: int = 0, stream=None,
                      keep_results: bool = False, autotune: bool = True,
                      clock=time.perf_counter, sleep=time.sleep) -> List[Result]:
    """The same requests served one plate at a time, in arrival order, with
    plain launches (each plate in its autotuned launch shape)."""
    reqs = list(requests)
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
    results: List[Optional[Result]] = [None] * len(reqs)
    t0 = clock()
    for i in order:
        r = reqs[i]
        now = clock() - t0
        if now < r.arrival:
            sleep(r.arrival - now)
        adm = clock() - t0
        s = slbm.Solver(r.plate, precision, device=device, stream=stream)
        if autotune:
            s.autotune()
        s.step(r.steps)
        diverged, u = _readout(s, keep_results)
        s.close()
        results[i] = Result(i, r.arrival, adm, clock() - t0, r.steps, r.plate.n_material, diverged, False, u)
    return results


def summary(results: List[Result]) -> dict:
    """Latency percentiles (s), queue wait, and aggregate throughput (MLUPS,
    material-site updates over the time from the start to the last result)."""
    done = [r for r in results if r is not None and not r.rejected]
    lat = np.array([r.latency for r in done])
    wait = np.array([r.wait for r in done])
    span = max(r.finished for r in done)
    work = sum(r.sites * r.steps for r in done)
    return {
        "requests": len(done),
        "rejected": sum(1 for r in results if r is not None and r.rejected),
        "diverged": sum(1 for r in done if r.diverged),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "mean_queue_wait_s": round(float(wait.mean()), 4),
        "makespan_s": round(span, 4),
        "aggregate_mlups": round(work / span / 1e6, 1),
    }
