"""Serving loop: continuous batching of plate solves on one GPU.

Requests arrive over time, each a plate and a number of steps.  A waiting
request is admitted into the resident batch (slbm_batch_add) as soon as its
device footprint fits the HBM budget, first come first served, and -- when a
cap is set -- as long as the material sites resident stay within it (enough
plates to fill the machine, not so many that every request shares it with
every other and finishes late).  With policy "swf" the waiting request with
the least work (sites x steps) goes first instead of the oldest.  Every
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
                 stream=None, launch=None, max_resident_sites: Optional[int] = None, policy: str = "fcfs",
                 xcd_group: int = 0):
        self.batch = slbm.Batch(budget_bytes, device=device, stream=stream)
        self.precision = precision
        self.chunk = int(chunk)
        self.max_sites = max_resident_sites
        if policy not in ("fcfs", "swf"):
            raise ValueError("policy must be 'fcfs' or 'swf'")
        self.policy = policy
        self.peak_bytes = 0
        self.peak_resident = 0
        if launch is not None:
            self.batch.set_launch(*launch)
        self.batch.set_xcd_group(xcd_group)

    def close(self):
        self.batch.close()

    def run(self, requests: Iterable[Request], keep_results: bool = False,
            clock=time.perf_counter, sleep=time.sleep) -> List[Result]:
        reqs = list(requests)
        nsites = [int(r.plate.n_material) for r in reqs]
        work = [n * r.steps for n, r in zip(nsites, reqs)]
        order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
        pending = collections.deque(order)
        waiting = collections.deque()
        resident = {}                     # slot -> (request index, admitted time)
        sites = 0                         # material sites resident
        results: List[Optional[Result]] = [None] * len(reqs)
        t0 = clock()
        while pending or waiting or resident:
            now = clock() - t0
            while pending and reqs[pending[0]].arrival <= now:
                waiting.append(pending.popleft())
            if self.policy == "swf" and len(waiting) > 1:
                waiting = collections.deque(sorted(waiting, key=lambda i: (work[i], reqs[i].arrival)))
            # admission in policy order while the head fits
            while waiting:
                i = waiting[0]
                r = reqs[i]
                if (self.max_sites is not None and resident
                        and sites + nsites[i] > self.max_sites):
                    break
                try:
                    slot = self.batch.add(r.plate, r.steps, self.precision)
                except slbm.SlbmError as e:
                    if e.code != -6:
                        raise
                    if not resident:
                        # larger than the whole budget: it can never run
                        waiting.popleft()
                        t = clock() - t0
                        results[i] = Result(i, r.arrival, t, t, r.steps, nsites[i], False, True)
                        continue
                    break
                waiting.popleft()
                resident[slot] = (i, clock() - t0)
                sites += nsites[i]
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
                sites -= nsites[i]
                diverged, u = _readout(self.batch.solver(slot), keep_results)
                self.batch.remove(slot)
                results[i] = Result(i, r.arrival, adm, clock() - t0, r.steps, nsites[i], diverged, False, u)
        return results


def run_one_at_a_time(requests: Iterable[Request], precision: str = "fp32", device: int = 0, stream=None,
                      keep_results: bool = False, autotune: bool = True, policy: str = "fcfs",
                      clock=time.perf_counter, sleep=time.sleep) -> List[Result]:
    """The same requests served one plate at a time with plain launches
    (each plate in its autotuned launch shape, or the library's default):
    the oldest waiting request first ("fcfs") or the one with the least work
    ("swf")."""
    if policy not in ("fcfs", "swf"):
        raise ValueError("policy must be 'fcfs' or 'swf'")
    reqs = list(requests)
    work = [int(r.plate.n_material) * r.steps for r in reqs]
    pending = collections.deque(sorted(range(len(reqs)), key=lambda i: reqs[i].arrival))
    waiting: List[int] = []
    results: List[Optional[Result]] = [None] * len(reqs)
    t0 = clock()
    while pending or waiting:
        now = clock() - t0
        while pending and reqs[pending[0]].arrival <= now:
            waiting.append(pending.popleft())
        if not waiting:
            sleep(max(0.0, reqs[pending[0]].arrival - now))
            continue
        i = min(waiting, key=lambda j: (work[j], reqs[j].arrival)) if policy == "swf" else waiting[0]
        waiting.remove(i)
        r = reqs[i]
        adm = clock() - t0
        s = slbm.Solver(r.plate, precision, device=device, stream=stream)
        if autotune:
            s.autotune()
        s.step(r.steps)
        diverged, u = _readout(s, keep_results)
        s.close()
        results[i] = Result(i, r.arrival, adm, clock() - t0, r.steps, int(r.plate.n_material), diverged, False, u)
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
