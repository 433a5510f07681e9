"""Batched path (slbm_batch_*): many plates in one launch per step, steps
replayed from a captured graph.  Every plate's result is checked against the
CPU reference element by element, and must be bit-identical to the same plate
run alone (the per-site arithmetic does not depend on the batch)."""
import dataclasses

import numpy as np
import pytest

from oracle import Oracle
from slbm_workloads import configs
from slbm_workloads import geometry as G
from test_gpu_parity import FP32_TOL, compare, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_04088_amd import slbm as S
    S.lib()
    return S


def small_plates(seed, count):
    """Uneven plates from the batched-workload generator, shrunk to test size."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(configs._random_plate(rng, area_lo=24 ** 2, area_hi=180 ** 2, load=1e-3, steps=0,
                                         name=f"small{seed}-{i}"))
    return out


def oracle_plates(seed, count):
    """Uneven plates of the batched-workload generator (0-3 holes, an edge
    crack with probability 1/2, mu ~ U[0.02, 0.08]) at test size, with
    lambda/mu redrawn in [0.5, 1] and the Neumann extrapolation order
    alternating between the two rules, and a last plate at lambda/mu = 1.8
    (tau_bar 0.6), whose traction-free walls grow a surface mode: it is
    compared over its first 40 steps only."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for i, p in enumerate(small_plates(seed, count)):
        last = i == count - 1
        lm = 1.8 if last else rng.uniform(0.5, 1.0)
        order = 0 if last else i % 2
        out.append(dataclasses.replace(p, lam=lm * p.mu, tau=configs.tau_for(lm), neumann_order=order,
                                       name=f"{p.name}-lm{lm:.2f}-o{order}"))
    return out


def alone(slbm, plate, steps, prec):
    s = slbm.Solver(plate, prec)
    s.step(steps)
    return s.displacement(), s.moments()[3]


def diverged(slbm, solver):
    """Whether the plate's state diverged (SLBM_E_DIVERGED at sync)."""
    try:
        solver.sync()
        return False
    except slbm.SlbmError as e:
        assert e.code == -4
        return True


def check_like_alone(slbm, plate, steps, prec, solver, u=None):
    """A batch plate's result against the same plate stepped alone: bit for
    bit while it stays finite; a plate whose state diverges (the random
    plates draw lambda/mu up to 2, whose free walls grow a surface mode) is
    flagged in both, its arithmetic stopped in the batch."""
    s = slbm.Solver(plate, prec)
    s.step(steps)
    if diverged(slbm, solver):
        assert diverged(slbm, s), plate.name
        return False
    assert not diverged(slbm, s), plate.name
    assert np.array_equal(solver.displacement() if u is None else u, s.displacement()), plate.name
    return True


@pytest.mark.parametrize("launch", [None, (6, 58)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_plates_match_their_solo_runs(slbm, prec, launch):
    """Step counts on both sides of the captured chunk and odd ones, in both
    launch modes (one step, or two steps per launch with single-step ends)."""
    plates = small_plates(3, 7)
    steps = [0, 1, 31, 32, 33, 70, 101]
    b = slbm.Batch(8 << 30)
    if launch:
        b.set_launch(*launch)
    slots = [b.add(p, n, prec) for p, n in zip(plates, steps)]
    for k in (5, 32, 1, 40, 64):        # chunks below, at and above the graph size
        b.step(k)
    b.sync()
    assert sorted(b.poll()) == sorted(slots)
    finite = 0
    for p, n, sl in zip(plates, steps, slots):
        s = b.solver(sl)
        assert s.time()[0] == n or diverged(slbm, s)
        if check_like_alone(slbm, p, n, prec, s):
            finite += 1
            u_ref, sig_ref = alone(slbm, p, n, prec)
            assert np.array_equal(b.displacement(sl), u_ref), p.name
            assert np.array_equal(s.moments()[3], sig_ref), p.name
    assert finite >= 4
    b.close()


@pytest.mark.parametrize("launch", [(6, 62), (6, 58), (10, 58)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_plates_match_the_reference(slbm, prec, launch):
    """Eight uneven random plates (holes, edge crack, both Neumann rules,
    lambda/mu in [0.5, 1] and one at 1.8) advanced together by uneven step
    chunks, each to its own step count: every plate's displacement, density,
    momentum, Poisson stress and Cauchy stress against the CPU reference
    (fp64 to 1e-12 against the extended-precision build, fp32 to 1e-4)."""
    plates = oracle_plates(21, 8)
    steps = [37, 64, 101, 150, 23, 211, 120, 40]
    b = slbm.Batch(8 << 30)
    b.set_launch(*launch)
    slots = [b.add(p, n, prec) for p, n in zip(plates, steps)]
    for sl in slots:
        # with two steps per launch every plate carries its tile lists
        assert b.solver(sl).boundary_lists()[0] == (launch[0] if launch[1] == 58 else 0)
    for k in (5, 32, 1, 40, 64, 128):        # chunks below, at and above the graph size, odd ones
        b.step(k)
    b.sync()
    assert sorted(b.poll()) == sorted(slots)
    for p, n, sl in zip(plates, steps, slots):
        s = b.solver(sl)
        assert s.time()[0] == n
        s.sync()
        ref = Oracle(p, extended=(prec == "fp64"))
        ref.step(n)
        e = compare(s, ref, prec)
        print(f"{p.name} {p.nx}x{p.ny} {n} steps {prec}: rel L2 u = {e:.2e}")
    b.close()


def test_batch_autotune_takes_real_steps(slbm):
    """slbm_batch_autotune times launch shapes with real steps: the plates
    advance by them, and their state equals the same number of steps taken
    alone; the shape it keeps is reported."""
    # lambda/mu <= 1 and the boundary-site Neumann rule: none diverges and is retired
    plates = [dataclasses.replace(p, neumann_order=0) for p in oracle_plates(7, 6)[:5]]
    b = slbm.Batch(8 << 30)
    slots = [b.add(p, 600, "fp32") for p in plates]
    rows, strip, group, us = b.autotune(600)
    assert strip in (58, 62) and group in (0, 8) and us > 0
    assert b.launch() == (rows, strip, group)
    taken = [b.solver(sl).time()[0] for sl in slots]
    assert len(set(taken)) == 1 and 0 < taken[0] <= 600
    b.step(33)
    for p, sl in zip(plates, slots):
        assert check_like_alone(slbm, p, taken[0] + 33, "fp32", b.solver(sl)), p.name
    b.close()


def test_batch_plate_handle_refuses_stepping(slbm):
    """A batch plate's handle is for readouts: stepping it, or changing its
    state or launch shape, would desynchronise the batch and is refused."""
    p = small_plates(8, 1)[0]
    b = slbm.Batch(8 << 30)
    sl = b.add(p, 10, "fp32")
    s = b.solver(sl)
    for call in (lambda: s.step(1), lambda: s.autotune(), lambda: s.set_launch(6, 58),
                 lambda: s.init_fields(), lambda: s.set_xcd_group(8)):
        with pytest.raises(slbm.SlbmError) as e:
            call()
        assert e.value.code == -1
    L = slbm.lib()
    assert L.slbm_step(s.h, 1) == -1 and L.slbm_destroy(s.h) == -1
    b.step(10)
    u_ref, _ = alone(slbm, p, 10, "fp32")
    assert np.array_equal(b.displacement(sl), u_ref)
    b.close()


@pytest.mark.parametrize("launch", [None, (4, 58)])
def test_continuous_batching_joins_and_leaves(slbm, launch):
    """Plates arrive while others are running and leave when done; each
    result is the same alone and in the mix."""
    plates = small_plates(5, 6)
    want = [45, 80, 33, 64, 100, 20]
    b = slbm.Batch(8 << 30)
    if launch:
        b.set_launch(*launch)
    live = {}
    arrivals = {0: [0, 1], 1: [2], 2: [3, 4], 4: [5]}
    finished = {}
    for tick in range(12):
        for i in arrivals.get(tick, []):
            live[b.add(plates[i], want[i], "fp32")] = i
        b.step(16)
        for sl in b.poll():
            i = live.pop(sl)
            s = b.solver(sl)
            finished[i] = (s.time()[0], b.displacement(sl), diverged(slbm, s))
            b.remove(sl)
    assert sorted(finished) == list(range(6))
    for i, (n, u, div) in finished.items():
        s = slbm.Solver(plates[i], "fp32")
        s.step(want[i])
        assert div == diverged(slbm, s), plates[i].name
        if not div:
            assert n == want[i]
            assert np.array_equal(u, s.displacement()), plates[i].name
    b.sync()                         # the removed plates' memory is reusable once their work has run
    assert b.bytes()[0] == 0
    b.close()


def test_batch_launch_shape_does_not_change_results(slbm):
    # lambda/mu <= 1 and the boundary-site Neumann rule: every plate stays finite
    plates = [dataclasses.replace(p, neumann_order=0) for p in oracle_plates(9, 5)[:4]]
    ref = None
    for rows, strip, group in ((2, 62, 0), (8, 64, 0), (5, 62, 0), (14, 64, 0), (14, 62, 0), (1, 58, 0),
                               (6, 58, 0), (10, 58, 0), (5, 62, 8), (6, 58, 8), (10, 58, 64), (3, 64, 2)):
        b = slbm.Batch(8 << 30)
        slots = [b.add(p, 50, "fp64") for p in plates]
        b.set_launch(rows, strip)
        b.set_xcd_group(group)
        b.step(50)
        us = [b.solver(sl).displacement() for sl in slots]
        if ref is None:
            ref = us
        else:
            for a, r in zip(us, ref):
                assert np.array_equal(a, r)
        b.close()


def test_budget_is_enforced(slbm):
    plates = small_plates(11, 3)
    b = slbm.Batch(1 << 20)      # 1 MiB: the first small plate fits, not all three
    ok, rejected = 0, 0
    for p in plates:
        try:
            b.add(p, 10, "fp32")
            ok += 1
        except slbm.SlbmError as e:
            assert e.code == -6
            rejected += 1
    assert rejected >= 1
    used, budget = b.bytes()
    assert used <= budget
    b.close()


def test_batch_divergence_is_per_plate(slbm):
    """One plate that blows up (lambda/mu = 2, traction-free, the paper's
    extrapolation) flags itself, is retired before its step count (its
    remaining steps set to zero), and leaves its neighbours' results intact."""
    n = 40
    bad = G.build_plate(n, n, lam=0.1, mu=0.05, tau=0.6, walls=G.edge_walls(n, n, 0, 0, 1, 1),
                        groups=[G.BCGroup(G.NEUMANN, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (0.0, 1e-4))],
                        neumann_order=1, name="unstable")
    # straight walls only, lambda = mu, boundary-site rule: stays finite over
    # thousands of steps (curved traction-free walls with small q grow slowly)
    good = configs.square_clamped_pulled(48)
    b = slbm.Batch(8 << 30)
    sb = b.add(bad, 20000, "fp32")
    sg = b.add(good, 4000, "fp32")
    for _ in range(4000 // 64 + 1):
        b.step(64)
    b.sync()
    assert sorted(b.poll()) == sorted([sb, sg])
    assert b.remaining(sb) == 0
    stopped = b.solver(sb).time()[0]
    assert stopped < 20000
    with pytest.raises(slbm.SlbmError) as e:
        b.solver(sb).sync()
    assert e.value.code == -4
    b.solver(sg).sync()
    u_ref, _ = alone(slbm, good, 4000, "fp32")
    assert np.array_equal(b.solver(sg).displacement(), u_ref)
    print(f"diverged plate retired after {stopped} of 20000 steps")
    b.close()


def test_empty_batch_is_a_no_op(slbm):
    """A batch with no plates steps, polls, autotunes and syncs as a no-op,
    before its first plate arrives and after its last one leaves; the plates
    in between, one of them asked for zero steps, give their solo results."""
    b = slbm.Batch(1 << 30)
    b.step(10)
    assert b.poll() == []
    b.sync()
    shape = b.launch()
    assert b.autotune(200) == (*shape, 0.0)          # nothing to time: the shape stays
    p, p0 = [dataclasses.replace(q, neumann_order=0) for q in oracle_plates(4, 3)[:2]]
    sl = b.add(p, 30, "fp32")
    sl0 = b.add(p0, 0, "fp32")                      # a plate asked for zero steps
    assert b.poll() == [sl0]
    b.step(40)
    assert sorted(b.poll()) == sorted([sl, sl0])
    assert check_like_alone(slbm, p, 30, "fp32", b.solver(sl), b.displacement(sl))
    assert check_like_alone(slbm, p0, 0, "fp32", b.solver(sl0), b.displacement(sl0))
    assert b.solver(sl0).time()[0] == 0
    b.remove(sl)
    b.remove(sl0)
    b.step(10)
    assert b.poll() == []
    b.sync()
    assert b.bytes()[0] == 0
    b.close()
