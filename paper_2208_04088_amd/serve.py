"""Serving loop: continuous batching of plate solves on one GPU.

Requests arrive over time, each a plate and a number of steps.  A waiting
request is admitted into the resident batch (slbm_batch_add) as soon as its
device footprint fits the HBM budget, first come first served, and -- when a
cap is set -- as long as the material sites resident stay within it (enough
plates to fill the machine, not so many that every request shares it with
every other and finishes late).  With policy "swf" the waiting request with
the least work (sites x steps) goes first instead of the oldest.  Every
resident plate is advanced together, one launch per step (or two) for all of
them, a round of steps at a time (each plate by at most its remaining steps).

The host never waits for the round it has just queued: after queuing round
r it reads back the plates that finished in round r - 1 (each readout waits
for that plate's last steps only, on the batch's side stream), removes them
and admits new requests, so the GPU runs round r meanwhile.  Plates whose
state overflowed are retired by the batch (SLBM_E_DIVERGED) and reported as
such, without taking their remaining steps.  All state stays on the device
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

# material-site updates per microsecond the batched kernel sustains (sizes a
# round of steps to a target duration)
RATE_SITES_PER_US = 40e3


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
    steps_taken: int = 0

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
    """Continuous batching under an HBM budget (bytes).

    chunk: steps per round (the least, with round_ms); round_ms: target GPU
    time of a round, from the resident sites; depth: rounds queued on the
    device at most; timing_stream: a torch stream (the batch's) on which to
    time the rounds, for the GPU-busy fraction."""

    def __init__(self, budget_bytes: int, precision: str = "fp32", chunk: int = 64, device: int = 0,
                 stream=None, launch=None, max_resident_sites: Optional[int] = None, policy: str = "fcfs",
                 xcd_group: int = 0, round_ms: Optional[float] = None, timing_stream=None, depth: int = 3):
        self.batch = slbm.Batch(budget_bytes, device=device, stream=stream)
        self.precision = precision
        self.chunk = int(chunk)
        self.round_ms = round_ms
        self.max_sites = max_resident_sites
        if policy not in ("fcfs", "swf"):
            raise ValueError("policy must be 'fcfs' or 'swf'")
        self.policy = policy
        self.peak_bytes = 0
        self.peak_resident = 0
        self.timing_stream = timing_stream
        self.depth = max(1, int(depth))
        self.gpu_busy_s = None
        self.gpu_span_s = None
        self.rounds = 0
        if launch is not None:
            self.batch.set_launch(*launch)
        self.batch.set_xcd_group(xcd_group)

    def close(self):
        self.batch.close()

    def _round_steps(self, sites: int) -> int:
        if not self.round_ms:
            return self.chunk
        steps = int(self.round_ms * 1e3 * RATE_SITES_PER_US / max(sites, 1))
        return max(self.chunk, min(4096, steps // 32 * 32))

    def run(self, requests: Iterable[Request], keep_results: bool = False,
            clock=time.perf_counter, sleep=time.sleep) -> List[Result]:
        reqs = list(requests)
        nsites = [int(r.plate.n_material) for r in reqs]
        work = [n * r.steps for n, r in zip(nsites, reqs)]
        order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
        pending = collections.deque(order)
        waiting = collections.deque()
        resident = {}                     # slot -> (request index, admitted time): still stepping
        finishing = {}                    # slot -> (request index, admitted time): steps all queued
        sites = 0                         # material sites of the plates still stepping
        results: List[Optional[Result]] = [None] * len(reqs)
        events = []
        t0 = clock()
        while pending or waiting or resident or finishing:
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
                    if not resident and not finishing:
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
            self.peak_resident = max(self.peak_resident, len(resident) + len(finishing))
            # queue the next round before touching the plates of the last one
            if resident:
                if self.timing_stream is not None:
                    import torch
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(self.timing_stream)
                self.batch.step(self._round_steps(sites))
                if self.timing_stream is not None:
                    e1.record(self.timing_stream)
                    events.append((e0, e1))
                self.rounds += 1
            # at most `depth` rounds in flight: the device has the next ones
            # queued while the host admits and reads out, and the host never
            # runs far ahead of what it has seen (plates found diverged are
            # retired within a few rounds)
            self.batch.wait(self.depth - 1)
            # results of the plates whose steps were all queued before this round
            for slot, (i, adm) in list(finishing.items()):
                r = reqs[i]
                sv = self.batch.solver(slot)
                diverged, u = _readout(sv, keep_results)
                taken = sv.time()[0]
                self.batch.remove(slot)
                del finishing[slot]
                results[i] = Result(i, r.arrival, adm, clock() - t0, r.steps, nsites[i], diverged, False, u,
                                    taken)
            for slot in self.batch.poll():
                if slot in resident:
                    finishing[slot] = resident.pop(slot)
                    sites -= nsites[finishing[slot][0]]
            if not resident and not finishing and pending and not waiting:
                sleep(max(0.0, reqs[pending[0]].arrival - (clock() - t0)))
        if events:
            import torch
            torch.cuda.synchronize()
            self.gpu_busy_s = sum(a.elapsed_time(b) for a, b in events) / 1e3
            self.gpu_span_s = events[0][0].elapsed_time(events[-1][1]) / 1e3
        return results


def run_one_at_a_time(requests: Iterable[Request], precision: str = "fp32", device: int = 0, stream=None,
                      keep_results: bool = False, autotune: bool = True, policy: str = "fcfs",
                      clock=time.perf_counter, sleep=time.sleep, check_every: int = 1024,
                      launch=None, xcd_group: int = 0) -> List[Result]:
    """The same requests served one plate at a time with plain launches
    (each plate in its autotuned launch shape, in `launch` = (rows, strip)
    with `xcd_group` when given, or the library's default):
    the oldest waiting request first ("fcfs") or the one with the least work
    ("swf").  A plate is checked for divergence every `check_every` steps
    and stopped when its state has overflowed, as the server retires it."""
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
        if launch is not None:
            s.set_launch(*launch)
            s.set_xcd_group(xcd_group)
        elif autotune:
            s.autotune()
        done = 0
        while done < r.steps:
            k = min(check_every, r.steps - done)
            s.step(k)
            done += k
            if done < r.steps:
                try:
                    s.sync()
                except slbm.SlbmError as e:
                    if e.code != -4:
                        raise
                    break
        diverged, u = _readout(s, keep_results)
        s.close()
        results[i] = Result(i, r.arrival, adm, clock() - t0, r.steps, int(r.plate.n_material), diverged, False, u,
                            done)
    return results


def summary(results: List[Result]) -> dict:
    """Latency percentiles (s), queue wait and aggregate throughput (MLUPS:
    material-site updates of the requests that completed, over the time from
    the start to the last result) of the completed requests; requests whose
    state overflowed are counted apart, with the steps they took."""
    served = [r for r in results if r is not None and not r.rejected]
    done = [r for r in served if not r.diverged]
    bad = [r for r in served if r.diverged]
    span = max(r.finished for r in served) if served else 0.0
    out = {
        "requests": len(done),
        "rejected": sum(1 for r in results if r is not None and r.rejected),
        "diverged": len(bad),
        "makespan_s": round(span, 4),
    }
    if done:
        lat = np.array([r.latency for r in done])
        wait = np.array([r.wait for r in done])
        out.update({
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "mean_queue_wait_s": round(float(wait.mean()), 4),
            "aggregate_mlups": round(sum(r.sites * r.steps for r in done) / span / 1e6, 1),
        })
    if bad:
        out["diverged_steps_taken_mean"] = round(float(np.mean([r.steps_taken for r in bad])), 1)
        out["diverged_detect_latency_p50_s"] = round(float(np.percentile([r.latency for r in bad], 50)), 4)
    return out
