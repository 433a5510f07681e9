"""slbm_displacement_device_noalloc: the displacement readout with no device
allocation (its density scratch is the library's static per-device array),
checked against slbm_displacement_device on the same state, on two calls in
a row, the second with a smaller plate; plates beyond the array are refused;
the call leaves no scratch behind (the handle's device bytes do not change)."""
import numpy as np
import pytest

from slbm_workloads import geometry as G
from test_gpu_parity import mixed_plate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_04088_amd import slbm as S
    S.lib()
    return torch, S


def readouts(torch, S, s):
    """The state's displacement through both device entry points, into torch memory."""
    n = s.plate.nx * s.plate.ny
    a = torch.full((2 * n,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((2 * n,), float("nan"), dtype=torch.float64, device="cuda")
    before = s.device_bytes()
    s.displacement_device_noalloc(b.data_ptr())
    s.sync()
    assert s.device_bytes() == before              # no scratch was allocated for the call
    s.displacement_device(a.data_ptr())
    s.sync()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_readout_equals_the_allocating_one(env, prec):
    torch, S = env
    big = mixed_plate(150, 97, seed=5, order=1)
    small = mixed_plate(40, 30, seed=9, order=0)
    periodic = mixed_plate(64, 40, seed=1, periodic=True)
    for plate, steps in ((big, 37), (small, 11), (periodic, 20)):   # each call smaller than the one before
        s = S.Solver(plate, prec)
        s.step(steps)
        a, b = readouts(torch, S, s)
        assert np.isfinite(b).all() and np.abs(b).max() > 0
        assert np.array_equal(a, b), plate.name
        assert np.array_equal(b.reshape(2, plate.ny, plate.nx), s.displacement()), plate.name
        s.close()


def test_noalloc_readout_of_a_batch_plate(env):
    torch, S = env
    plates = [mixed_plate(90, 60, seed=11, order=1), mixed_plate(50, 35, seed=12, order=0)]
    b = S.Batch(1 << 30)
    slots = [b.add(p, n, "fp32") for p, n in zip(plates, (40, 23))]
    b.step(40)
    for p, sl in zip(plates, slots):
        x, y = readouts(torch, S, b.solver(sl))
        assert np.array_equal(x, y), p.name
    b.close()


def test_noalloc_readout_refuses_plates_beyond_the_static_array(env):
    torch, S = env
    # 1 x 300000 sites: padded plane 128 x 300002 = 38.4M sites > 18874368
    p = G.build_plate(1, 300000, lam=0.05, mu=0.05, tau=0.55, walls=[G.HLine(-0.5, 0), G.HLine(299999.5, 0)],
                      groups=[G.BCGroup(G.NEUMANN, (0.0, 0.0))], periodic_x=True, neumann_order=0)
    s = S.Solver(p, "fp32")
    u = torch.zeros(2 * 300000, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SlbmError) as e:
        s.displacement_device_noalloc(u.data_ptr())
    assert e.value.code == -1 and "static readout scratch" in str(e.value)
    with pytest.raises(S.SlbmError) as e:
        s.displacement_device_noalloc(0)
    assert e.value.code == -1
    s.close()
