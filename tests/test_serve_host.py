"""Host logic of the serving loop without a GPU: a stand-in for the batch
records what the loop asks of it (admission against the byte budget and the
resident-sites cap, policy order, retirement), with a simulated clock that
advances with the steps taken."""
import types

import numpy as np
import pytest

from paper_2208_04088_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBatch:
    """Bytes per plate = 100 x sites; one step costs 1e-5 s per resident site."""

    def __init__(self, budget, clock):
        self.budget, self.clock = budget, clock
        self.slots = {}
        self.next = 0
        self.used = 0
        self.order = []
        self.max_sites_seen = 0
        self.steps_called = []

    def add(self, plate, steps, prec):
        need = 100 * plate.n_material
        if self.used + need > self.budget:
            raise serve.slbm.SlbmError(-6, "budget")
        s = self.next
        self.next += 1
        self.slots[s] = [plate, steps, need]
        self.used += need
        self.order.append(plate.name)
        # sites of the plates still stepping (finished ones wait for their readout)
        self.max_sites_seen = max(self.max_sites_seen,
                                  sum(p.n_material for p, r, _ in self.slots.values() if r > 0))
        return s

    def step(self, k):
        sites = sum(p.n_material for p, r, _ in self.slots.values() if r > 0)
        self.clock.t += 1e-5 * sites * k
        for v in self.slots.values():
            v[1] = max(0, v[1] - k)
        self.steps_called.append(k)

    def sync(self):
        pass

    def wait(self, n):
        pass

    def poll(self):
        return [s for s, v in self.slots.items() if v[1] == 0]

    def solver(self, slot):
        plate, rem, _ = self.slots[slot]
        return types.SimpleNamespace(sync=lambda: None, displacement=lambda: np.zeros(1),
                                     time=lambda: (0, 0.0))

    def remove(self, slot):
        self.used -= self.slots.pop(slot)[2]

    def bytes(self):
        return self.used, self.budget

    def set_launch(self, *a):
        pass

    def set_xcd_group(self, g):
        self.xcd_group = g

    def close(self):
        pass


class P:
    def __init__(self, name, n):
        self.name, self.n_material = name, n


def server(monkeypatch, budget, **kw):
    clock = FakeClock()
    made = {}

    def mk(b, device=0, stream=None):
        made["b"] = FakeBatch(b, clock)
        return made["b"]

    monkeypatch.setattr(serve.slbm, "Batch", mk)
    srv = serve.Server(budget, chunk=10, **kw)
    return srv, made["b"], clock


def trace():
    # (arrival, sites, steps): everything arrives at once except the last
    spec = [(0.0, 1000, 50), (0.0, 4000, 10), (0.0, 500, 200), (0.0, 2000, 20), (0.5, 100, 10)]
    return [serve.Request(a, P(f"r{i}", n), s) for i, (a, n, s) in enumerate(spec)]


def test_fcfs_admits_in_arrival_order_within_the_budget(monkeypatch):
    srv, b, clock = server(monkeypatch, budget=100 * 5000)
    res = srv.run(trace(), clock=clock, sleep=clock.sleep)
    assert all(r is not None and not r.rejected for r in res)
    assert b.order == ["r0", "r1", "r2", "r3", "r4"]
    assert srv.peak_bytes <= 100 * 5000
    for r in res:
        assert r.arrival <= r.admitted <= r.finished


def test_cap_limits_resident_sites(monkeypatch):
    srv, b, clock = server(monkeypatch, budget=10 ** 12, max_resident_sites=4500)
    srv.run(trace(), clock=clock, sleep=clock.sleep)
    assert b.max_sites_seen <= 4500


def test_least_work_first_order(monkeypatch):
    srv, b, clock = server(monkeypatch, budget=10 ** 12, max_resident_sites=1, policy="swf")
    srv.run(trace(), clock=clock, sleep=clock.sleep)
    # one at a time (cap 1 site), work = sites x steps among those waiting:
    # r1 4e4 and r3 4e4 (tie: the earlier request), r0 5e4, r2 1e5; r4 (1e3)
    # arrives at 0.5 s while r3 runs (r1 takes 0.4 s, r3 another 0.4 s) and
    # goes next
    assert b.order == ["r1", "r3", "r4", "r0", "r2"]


def test_plate_larger_than_the_budget_is_rejected(monkeypatch):
    srv, b, clock = server(monkeypatch, budget=100 * 1500)
    res = srv.run(trace(), clock=clock, sleep=clock.sleep)
    rejected = sorted(r.index for r in res if r.rejected)
    assert rejected == [1, 3]
    assert all(not r.rejected for i, r in enumerate(res) if i not in (1, 3))


def test_summary_percentiles():
    rs = [serve.Result(i, 0.0, 0.0, float(i + 1), 10, 100, False) for i in range(100)]
    st = serve.summary(rs)
    assert st["p50_latency_s"] == pytest.approx(50.5)
    assert st["p99_latency_s"] == pytest.approx(99.01)
    assert st["aggregate_mlups"] == pytest.approx(100 * 10 * 100 / 100 / 1e6, abs=0.1)


def test_summary_counts_diverged_requests_apart():
    """Latency and throughput are over the requests that completed; those
    whose state overflowed are counted with the steps they took."""
    rs = [serve.Result(i, 0.0, 0.0, float(i + 1), 10, 100, False) for i in range(4)]
    rs.append(serve.Result(4, 0.0, 0.0, 9.0, 1000, 10 ** 6, True, steps_taken=64))
    st = serve.summary(rs)
    assert st["requests"] == 4 and st["diverged"] == 1
    assert st["p99_latency_s"] == pytest.approx(3.97)
    assert st["makespan_s"] == 9.0
    assert st["aggregate_mlups"] == pytest.approx(4 * 100 * 10 / 9.0 / 1e6, abs=1e-3)
    assert st["diverged_steps_taken_mean"] == 64


def test_next_round_is_queued_before_readout(monkeypatch):
    """The loop queues round r + 1 before it reads back the plates that
    finished in round r, so the device is never idle for a readout."""
    srv, b, clock = server(monkeypatch, budget=10 ** 12)
    calls = []
    real_step, real_solver = b.step, b.solver

    def step(k):
        calls.append(("step", k))
        real_step(k)

    def solver(slot):
        calls.append(("readout", slot))
        return real_solver(slot)

    b.step, b.solver = step, solver
    spec = [(0.0, 100, 10), (0.0, 100, 40)]
    srv.run([serve.Request(a, P(f"r{i}", n), s) for i, (a, n, s) in enumerate(spec)], clock=clock,
            sleep=clock.sleep)
    # r0 finishes in the first round; its readout comes after the second is queued
    first_readout = next(i for i, c in enumerate(calls) if c[0] == "readout")
    assert [c[0] for c in calls[:first_readout]] == ["step", "step"]


def test_round_length_follows_the_resident_sites(monkeypatch):
    srv, b, clock = server(monkeypatch, budget=10 ** 12, round_ms=10.0)
    spec = [(0.0, 10 ** 6, 2000)]
    srv.run([serve.Request(a, P(f"r{i}", n), s) for i, (a, n, s) in enumerate(spec)], clock=clock,
            sleep=clock.sleep)
    # 10 ms at 40e3 sites per microsecond over 1e6 sites: 400 steps a round
    assert b.steps_called[0] == 384


def test_empty_trace_and_zero_step_request(monkeypatch):
    """No requests: nothing is admitted and the summary reports none.  A
    request for zero steps completes with its rest state, alongside others."""
    srv, b, clock = server(monkeypatch, budget=10 ** 12)
    assert srv.run([], clock=clock, sleep=clock.sleep) == []
    assert b.order == []
    st = serve.summary([])
    assert st["requests"] == 0 and st["diverged"] == 0 and st["makespan_s"] == 0.0
    srv, b, clock = server(monkeypatch, budget=10 ** 12)
    reqs = [serve.Request(0.0, P("zero", 300), 0), serve.Request(0.0, P("ten", 300), 10)]
    res = srv.run(reqs, clock=clock, sleep=clock.sleep)
    assert [r.rejected or r.diverged for r in res] == [False, False]
    assert all(r.arrival <= r.admitted <= r.finished for r in res)
    assert serve.summary(res)["requests"] == 2
