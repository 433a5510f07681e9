"""HIP path (through the C ABI) against the CPU reference, element by element.

Tolerances: the fp64 path must match to 1e-12 relative (of the field's
largest value, and in relative L2); the fp32 path (fp32 populations and
arithmetic, fp64 displacement) to 1e-4 relative L2 on displacement, the
accuracy the method has to hold after 10k steps.
"""
import math
import os

import numpy as np
import pytest

from slbm_workloads import configs
from slbm_workloads import geometry as G
from oracle import Oracle

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def slbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_04088_amd import slbm as S
    S.lib()
    return S


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def compare(solver, ref, prec, what="all"):
    u, u_ref = solver.displacement(), ref.displacement()
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    assert np.isfinite(u).all()
    e = rel_l2(u, u_ref)
    assert e <= tol, f"u rel L2 {e:.3e} > {tol}"
    if prec == "fp64":
        scale = np.abs(u_ref).max()
        assert np.abs(u - u_ref).max() <= 4 * tol * scale
    if what == "all":
        for a, b, name in zip(solver.moments(), ref.moments(), ("rho", "j", "P", "sigma")):
            if name == "rho":
                a, b = a - 1.0 * (b != 0), b - 1.0 * (b != 0)   # compare the deviation from rest
            sc = np.abs(b).max()
            if sc < 1e-14:
                # the field is zero up to rounding in the reference
                assert np.abs(a).max() < 1e-12, f"{name}: {np.abs(a).max():.3e} where the reference is 0"
                continue
            d = np.abs(a - b).max() / sc
            lim = 4 * FP64_TOL if prec == "fp64" else 1e-3
            assert d <= lim, f"{name}: max deviation {d:.3e} of scale {sc:.3e}"
    return e


def mixed_plate(nx, ny, seed, order=0, periodic=False):
    """Straight edges (Dirichlet and Neumann, step and ramp), a curved hole,
    an edge crack, corners, body force."""
    rng = np.random.default_rng(seed)
    mu = 0.05
    groups = [G.BCGroup(G.DIRICHLET, (0.0, 0.0)),
              G.BCGroup(G.NEUMANN, (1e-3 * mu, 2e-4 * mu)),
              G.BCGroup(G.NEUMANN, (0.0, 0.0)),
              G.BCGroup(G.NEUMANN, (0.0, -5e-4 * mu), G.PROFILE_RAMP, 40.0),
              G.BCGroup(G.DIRICHLET, (1e-4, -2e-4), G.PROFILE_RAMP, 30.0)]
    if periodic:
        # the body force presses the material against a clamped hole; a
        # second, smaller hole moves (ramped curved Dirichlet wall)
        walls = [G.Circle(nx * 0.45, ny * 0.55, min(nx, ny) * 0.18, 0),
                 G.Circle(nx * 0.8, ny * 0.25, min(nx, ny) * 0.1, 4)]
        return G.build_plate(nx, ny, lam=0.04, mu=mu, tau=0.55, walls=walls, groups=groups,
                             force=(1e-6, -2e-6), periodic_x=True, periodic_y=True,
                             neumann_order=order, name=f"periodic{nx}x{ny}")
    walls = G.edge_walls(nx, ny, left=0, right=1, bottom=3, top=4)
    walls.append(G.Circle(nx * 0.62 + rng.uniform(-1, 1), ny * 0.5 + rng.uniform(-1, 1),
                          min(nx, ny) * 0.17, 2))
    walls.append(G.HLine(math.floor(ny * 0.3) + 0.5, 2, x_lo=-0.5, x_hi=nx * 0.3 - 0.5))
    return G.build_plate(nx, ny, lam=0.045, mu=mu, tau=0.55, walls=walls, groups=groups,
                         force=(1e-6, 0.0), neumann_order=order, name=f"mixed{nx}x{ny}")


# --------------------------------------------------------------- small --

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("shape", [(70, 45), (130, 67)])
def test_mixed_plate_matches_reference(slbm, prec, order, shape):
    """Several strips and row segments, a ragged last strip, every link kind."""
    p = mixed_plate(*shape, seed=shape[0], order=order)
    steps = 150
    ref = Oracle(p, extended=True)
    ref.step(steps)
    s = slbm.Solver(p, prec)
    s.step(steps)
    s.sync()
    compare(s, ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_periodic_plate_with_hole_and_force(slbm, prec):
    p = mixed_plate(64, 40, seed=1, periodic=True)
    ref = Oracle(p, extended=True)
    ref.step(120)
    s = slbm.Solver(p, prec)
    s.step(120)
    s.sync()
    compare(s, ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_initial_fields_match_reference(slbm, prec):
    """slbm_init_fields: the equilibrium of given density, velocity, stress
    and displacement fields, then stepping."""
    p = mixed_plate(66, 50, seed=3, order=0)
    rng = np.random.default_rng(7)
    m = p.mask.astype(float)
    yy, xx = np.mgrid[0:p.ny, 0:p.nx]
    rho = 1.0 + 1e-3 * np.sin(xx / 7.0) * np.cos(yy / 5.0)
    vel = 1e-3 * np.stack([np.sin(yy / 9.0), np.cos(xx / 6.0)]) * m
    sig = 1e-5 * rng.standard_normal((3, p.ny, p.nx)) * m
    u0 = 1e-2 * rng.standard_normal((2, p.ny, p.nx)) * m
    ref = Oracle(p, extended=True)
    ref.init_fields(rho, vel, sig, u0)
    s = slbm.Solver(p, prec)
    s.init_fields(rho, vel, sig, u0)
    compare(s, ref, prec)          # the state itself, before any step
    ref.step(60)
    s.step(60)
    compare(s, ref, prec)


# ----------------------------------------------------- paper scale --

@pytest.mark.parametrize("c2_ratio", [3.0, 2.8])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paper_hole_plate_full_run(slbm, c2_ratio, prec):
    """The paper's plate with a circular hole (section 5.1) at its own size,
    80 x 80, ramped tension, the paper's Neumann rule, to t = 2 l/c_s."""
    p = configs.paper_hole_plate(c2_ratio)
    ref = Oracle(p, extended=True)
    ref.step(p.steps)
    s = slbm.Solver(p, prec)
    s.step(p.steps)
    s.sync()
    compare(s, ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paper_center_crack_full_run(slbm, prec):
    """The paper's stationary crack (section 5.2): 400 x 400, a centred crack
    of 100 cells whose faces are suddenly pushed apart, the paper's Neumann
    rule, to t = 2 l_c/c_d.  The faces open: the left face moves to -x, the
    right one to +x.  The fp64 reference is the extended-precision build: the
    plain fp64 one (unshifted populations) already differs from it by ~1e-11
    at the end of this run."""
    p = configs.paper_center_crack()
    ref = Oracle(p, extended=True)
    ref.step(p.steps)
    s = slbm.Solver(p, prec)
    s.step(p.steps)
    s.sync()
    compare(s, ref, prec)
    u = s.displacement()
    xc = (p.nx - 1) / 2.0
    ymid = p.ny // 2
    assert u[0, ymid, int(np.floor(xc))] < 0 < u[0, ymid, int(np.ceil(xc))]


def test_square_config_fp64_full_length(slbm):
    """128 x 128 plate, left edge clamped, right edge pulled, 2000 steps (fp64)."""
    p = configs.square_clamped_pulled()
    ref = Oracle(p, extended=True)
    ref.step(p.steps)
    s = slbm.Solver(p, "fp64")
    s.step(p.steps)
    s.sync()
    e = compare(s, ref, "fp64")
    print(f"square128 fp64 {p.steps} steps: rel L2 u = {e:.3e}")


@pytest.mark.slow
def test_square_config_fp64_10k_steps(slbm):
    """The fp64 path over 10^4 steps of the 128 x 128 plate: displacement and
    moments within 1e-12 of the extended-precision reference."""
    p = configs.square_clamped_pulled(steps=10000)
    ref = Oracle(p, extended=True)
    ref.step(p.steps)
    s = slbm.Solver(p, "fp64")
    s.step(p.steps)
    s.sync()
    e = compare(s, ref, "fp64")
    print(f"square128 fp64 {p.steps} steps: rel L2 u = {e:.3e}")


def test_square_config_fp32_10k_steps(slbm):
    """Same plate in fp32 for 10k steps: displacement within 1e-4 relative L2."""
    p = configs.square_clamped_pulled(steps=10000)
    ref = Oracle(p)
    ref.step(p.steps)
    s = slbm.Solver(p, "fp32")
    s.step(p.steps)
    s.sync()
    e = compare(s, ref, "fp32", what="u")
    print(f"square128 fp32 10000 steps: rel L2 u = {e:.3e}")


# ------------------------------------------------------ launch shapes --

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_result_does_not_depend_on_launch_shape(slbm, prec):
    """Every site's arithmetic is independent of how rows and columns are
    split into tiles and how tiles are dealt to the XCDs, so any launch shape
    and XCD map give bit-identical state; shapes and groups beyond the limits
    are refused."""
    p = mixed_plate(150, 97, seed=5, order=1)
    out = []
    for seg, strip, group in ((1, 62, 0), (3, 64, 0), (8, 62, 0), (14, 64, 0), (14, 62, 0), (2, 64, 0),
                              (0, 0, 0), (1, 58, 0), (6, 58, 0), (10, 58, 0), (3, 62, 8), (1, 58, 1),
                              (6, 58, 8), (10, 58, 64), (2, 64, 4)):
        s = slbm.Solver(p, prec)
        s.set_launch(seg, strip)
        s.set_xcd_group(group)
        assert s.launch() == (seg, strip, group)
        s.step(37)
        out.append((s.displacement(), s.moments()[2]))
    for u, P in out[1:]:
        assert np.array_equal(u, out[0][0])
        assert np.array_equal(P, out[0][1])
    s = slbm.Solver(p, prec)
    for seg, strip in ((15, 62), (15, 64), (11, 58), (-1, 62), (4, 63)):
        with pytest.raises(slbm.SlbmError) as e:
            s.set_launch(seg, strip)
        assert e.value.code == -1
    for group in (-1, 3, 65, 128):
        with pytest.raises(slbm.SlbmError) as e:
            s.set_xcd_group(group)
        assert e.value.code == -1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["periodic", "init_fields", "odd_steps"])
def test_two_steps_per_launch_match_single_steps(slbm, prec, case):
    """The two-steps-per-launch kernel keeps the first step's populations in
    LDS and takes the second from there: the state must be bit-identical to
    single steps -- periodic plates, a start from slbm_init_fields (the first
    step reads in place), and an odd step count (the last step single)."""
    if case == "periodic":
        p, n = mixed_plate(64, 40, seed=1, periodic=True), 40
    else:
        p, n = mixed_plate(130, 67, seed=2, order=1), (41 if case == "odd_steps" else 30)
    out = []
    for shape in ((6, 62), (6, 58), (2, 58), (10, 58)):
        s = slbm.Solver(p, prec)
        if case == "init_fields":
            yy, xx = np.mgrid[0:p.ny, 0:p.nx]
            vel = 1e-4 * np.stack([np.sin(yy / 5.0), np.cos(xx / 7.0)]) * p.mask
            s.init_fields(vel=vel)
        s.set_launch(*shape)
        s.step(n)
        s.sync()
        assert s.time()[0] == n
        out.append((s.displacement(), s.moments()))
    for u, m in out[1:]:
        assert np.array_equal(u, out[0][0])
        for a, b in zip(m, out[0][1]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["mixed", "mixed_order1", "periodic", "small_periodic", "big_hole"])
def test_tile_lists_match_site_by_site_rules(slbm, prec, case):
    """With strip 58 the library lists each tile's cut links and the tile
    evaluates their rules together (first step from global memory, second
    from LDS) instead of site by site; the inputs of every rule value are the
    same, so the state must be bit-identical to single steps (which take the
    rules site by site) -- edges, corners, a crack, a curved hole, step and
    ramped Dirichlet and Neumann groups, both extrapolation orders, periodic
    axes whose tile footprints wrap (a plate narrower than a strip), and a hole
    wider than a strip, whose tiles without material outputs are skipped."""
    if case == "big_hole":
        p, n = configs.hole_plate(200, 80.0, lam=0.05, tau=0.55), 41
    elif case == "periodic":
        p, n = mixed_plate(64, 40, seed=1, periodic=True), 41
    elif case == "small_periodic":
        p = G.build_plate(40, 23, lam=0.06, mu=0.05, tau=0.6, periodic_x=True,
                          walls=[G.HLine(-0.5, 0), G.HLine(22.5, 1), G.Circle(20.0, 11.0, 5.0, 1)],
                          groups=[G.BCGroup(G.DIRICHLET, (0.0, 0.0)),
                                  G.BCGroup(G.NEUMANN, (3e-5, 1e-5), G.PROFILE_RAMP, 20.0)],
                          neumann_order=1)
        n = 40
    else:
        p, n = mixed_plate(150, 97, seed=5, order=1 if case == "mixed_order1" else 0), 41
    ref = slbm.Solver(p, prec)
    ref.set_launch(6, 62)
    ref.step(n)
    for rows in (1, 4, 10):
        s = slbm.Solver(p, prec)
        s.set_launch(rows, 58)
        built, records, most = s.boundary_lists()
        assert built == rows and records > 0 and 0 < most <= min(576, 64 * (rows + 6)), (built, records, most)
        s.step(n)
        s.sync()
        assert np.array_equal(s.displacement(), ref.displacement())
        for a, b in zip(s.moments(), ref.moments()):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plate_too_dense_for_tile_lists(slbm, prec):
    """A plate cut into two-row strips by full-width cracks has more cut links
    per tile than a tile's LDS takes: no lists are kept, the two-step kernel
    takes the rules site by site, and the state still matches single steps
    and the CPU reference."""
    nx, ny = 70, 24
    walls = G.edge_walls(nx, ny, left=0, right=1, bottom=1, top=1)
    walls += [G.HLine(y + 0.5, 1, x_lo=-0.5, x_hi=nx - 0.5) for y in range(1, ny - 2, 2)]
    p = G.build_plate(nx, ny, lam=0.04, mu=0.05, tau=0.55, walls=walls,
                      groups=[G.BCGroup(G.DIRICHLET, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (2e-5, 0.0))],
                      neumann_order=0)
    s = slbm.Solver(p, prec)
    s.set_launch(10, 58)
    assert s.boundary_lists() == (0, 0, 0)
    s.step(30)
    one = slbm.Solver(p, prec)
    one.set_launch(6, 62)
    one.step(30)
    assert np.array_equal(s.displacement(), one.displacement())
    ref = Oracle(p, extended=True)
    ref.step(30)
    compare(s, ref, prec)


@pytest.mark.parametrize("shape", [(1, 7), (2, 2), (3, 5), (61, 9), (62, 3), (63, 4), (64, 65), (124, 2), (125, 33)])
def test_small_and_ragged_grids(slbm, shape):
    """Degenerate and ragged sizes around the 62-column strip and the 64-element pitch."""
    nx, ny = shape
    p = G.build_plate(nx, ny, lam=0.06, mu=0.05, tau=0.6, periodic_x=True,
                      walls=[G.HLine(-0.5, 0), G.HLine(ny - 0.5, 1)],
                      groups=[G.BCGroup(G.DIRICHLET, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (3e-5, 1e-5))],
                      neumann_order=0)
    ref = Oracle(p, extended=True)
    ref.step(40)
    s = slbm.Solver(p, "fp64")
    s.step(40)
    compare(s, ref, "fp64")
    s2 = slbm.Solver(p, "fp64")
    s2.set_launch(3, 58)                 # two steps per launch
    s2.step(40)
    compare(s2, ref, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_steps_and_rest_state(slbm, prec):
    """Zero steps: the rest state, whose readout already carries the S/2
    part of j from the body force."""
    p = mixed_plate(40, 30, seed=9)
    s = slbm.Solver(p, prec)
    s.step(0)
    assert s.time()[0] == 0
    compare(s, Oracle(p, extended=True), prec)


def islands_plate(nx, ny, sites, groups, pick, q=0.5, order=0):
    """Islands of material in a periodic void (sites: (x, y)); every link from
    an island site into the void is cut at q, with the link's own direction
    as the outward normal and group pick(k) for direction k.  Links whose
    site behind is void are thin (the rules then take q = 1/2 throughout).
    The library refuses a site whose 8 links are all cut, so every island
    site keeps a neighbour."""
    mask = np.zeros((ny, nx), np.uint8)
    for x, y in sites:
        mask[y, x] = 1
    recs = []
    for x, y in sites:
        for k in range(1, 9):
            if mask[(y + G.CY[k]) % ny, (x + G.CX[k]) % nx]:
                continue
            c = np.array([G.CX[k], G.CY[k]], dtype=float)
            recs.append((y * nx + x, k, q, pick(k), -1, tuple(c / np.linalg.norm(c)), (0.0, 0.0)))
    links = np.array(recs, dtype=G.LINK_DTYPE).reshape(-1)
    return G.Plate(nx, ny, 0.05, 0.05, 1.0, 0.55, mask, links, list(groups), periodic_x=True, periodic_y=True,
                   name=f"islands{nx}x{ny}", neumann_order=order)


# pairs along an axis and a diagonal, an L, a 2 x 2 block and a line one site thick
ISLANDS = [(2, 2), (3, 2), (6, 1), (7, 2), (10, 4), (11, 4), (10, 5), (2, 6), (3, 6), (2, 7), (3, 7)] + \
          [(x, 9) for x in range(5, 12)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plate_without_material(slbm, prec):
    """An empty plate (every site void, no links) steps in both launch forms
    and reads out zeros, as the reference does."""
    p = islands_plate(70, 13, [], [G.BCGroup(G.NEUMANN)], lambda k: 0)
    assert p.n_material == 0 and len(p.links) == 0
    ref = Oracle(p, extended=True)
    ref.step(20)
    for shape in (None, (3, 58)):
        s = slbm.Solver(p, prec)
        if shape:
            s.set_launch(*shape)
        s.step(20)
        s.sync()
        assert not np.any(s.displacement())
        compare(s, ref, prec)
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("q", [0.5, 0.3])
def test_islands_with_moving_walls(slbm, prec, q):
    """Islands of one to seven sites carried by moving Dirichlet walls on
    every link (thin links throughout), 60 steps, in both launch forms."""
    p = islands_plate(13, 11, ISLANDS, [G.BCGroup(G.DIRICHLET, (1e-4, -2e-4))], lambda k: 0, q=q)
    ref = Oracle(p, extended=True)
    ref.step(60)
    for shape in (None, (3, 58)):
        s = slbm.Solver(p, prec)
        if shape:
            s.set_launch(*shape)
        s.step(60)
        compare(s, ref, prec)
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [0, 1])
def test_loaded_islands_few_steps(slbm, prec, order):
    """Islands with clamped links facing +x and loaded Neumann links
    elsewhere.  Free islands are violently unstable under the Neumann rule
    (rounding noise grows about 1.8-fold per step), so the comparison stops
    after 6 steps, while the state is still small."""
    groups = [G.BCGroup(G.DIRICHLET), G.BCGroup(G.NEUMANN, (3e-5, 1e-5))]
    p = islands_plate(13, 11, ISLANDS, groups, lambda k: 0 if G.CX[k] > 0 else 1, q=0.4, order=order)
    ref = Oracle(p, extended=True)
    ref.step(6)
    s = slbm.Solver(p, prec)
    s.step(6)
    compare(s, ref, prec)
    s.close()


# ----------------------------------------------------- state handling --

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpoint_resume_is_bitwise(slbm, prec):
    p = mixed_plate(90, 60, seed=11, order=1)
    a = slbm.Solver(p, prec)
    a.step(80)
    ua = a.displacement()
    b = slbm.Solver(p, prec)
    b.step(40)
    buf = b.save()
    c = slbm.Solver(p, prec)
    c.load(buf)
    assert c.time()[0] == 40
    c.step(40)
    assert np.array_equal(c.displacement(), ua)


def test_divergence_is_reported(slbm):
    """lambda/mu = 2 with traction-free walls and the paper's extrapolation
    is linearly unstable; the non-finite guard must catch the blow-up."""
    n = 40
    p = G.build_plate(n, n, lam=0.1, mu=0.05, tau=0.6, walls=G.edge_walls(n, n, 0, 0, 1, 1),
                      groups=[G.BCGroup(G.NEUMANN, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (0.0, 1e-4))],
                      neumann_order=1)
    s = slbm.Solver(p, "fp32")
    s.step(3000)
    with pytest.raises(slbm.SlbmError) as e:
        s.sync()
    assert e.value.code == -4


def test_displacement_to_device_memory(slbm):
    import torch
    p = mixed_plate(70, 40, seed=13)
    stream = torch.cuda.Stream()
    assert stream.cuda_stream != 0
    s = slbm.Solver(p, "fp32", stream=stream.cuda_stream)
    s.step(30)
    with torch.cuda.stream(stream):
        t = torch.empty((2, p.ny, p.nx), dtype=torch.float64, device="cuda")
    s.displacement_device(t.data_ptr())
    stream.synchronize()
    assert np.array_equal(t.cpu().numpy(), s.displacement())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_moments_to_device_memory(slbm, prec):
    """slbm_moments_device writes what slbm_moments returns: the same doubles
    (dtype fp64), or those doubles rounded to float (dtype fp32), on the
    handle's stream; NULL pointers skip their fields."""
    import torch
    p = mixed_plate(70, 40, seed=13)
    stream = torch.cuda.Stream()
    s = slbm.Solver(p, prec, stream=stream.cuda_stream)
    s.step(30)
    ref = s.moments()
    for dt, tdt in (("fp64", torch.float64), ("fp32", torch.float32)):
        with torch.cuda.stream(stream):
            t = [torch.full(sh, 7.0, dtype=tdt, device="cuda")
                 for sh in ((p.ny, p.nx), (2, p.ny, p.nx), (3, p.ny, p.nx), (3, p.ny, p.nx))]
        s.moments_device(*[x.data_ptr() for x in t], dtype=dt)
        stream.synchronize()
        for got, want in zip(t, ref):
            w = want.astype(np.float32) if dt == "fp32" else want
            assert np.array_equal(got.cpu().numpy(), w)
        with torch.cuda.stream(stream):
            only_j = torch.full((2, p.ny, p.nx), 7.0, dtype=tdt, device="cuda")
        s.moments_device(0, only_j.data_ptr(), 0, 0, dtype=dt)
        stream.synchronize()
        w = ref[1].astype(np.float32) if dt == "fp32" else ref[1]
        assert np.array_equal(only_j.cpu().numpy(), w)


# ------------------------------------------------------- full sizes --

def rigid_part(d, mask):
    """Least-squares rigid-body displacement (translation + infinitesimal
    rotation) contained in a displacement difference d [2, ny, nx]."""
    ny, nx = mask.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    w = mask.astype(bool)
    n = int(w.sum())
    A = np.zeros((2 * n, 3))
    A[:n, 0] = 1.0
    A[n:, 1] = 1.0
    A[:n, 2] = -(yy[w] - ny / 2)
    A[n:, 2] = xx[w] - nx / 2
    c, *_ = np.linalg.lstsq(A, np.concatenate([d[0][w], d[1][w]]), rcond=None)
    r = A @ c
    out = np.zeros_like(d)
    out[0][w], out[1][w] = r[:n], r[n:]
    return out


@pytest.mark.slow
def test_crack_config_fp32_full_length(slbm):
    """1024 x 512 edge-crack plate, fp32 populations, fp64 displacement, 10k
    steps, against the fp64 reference: relative L2 of the displacement and of
    the stress within 1e-4.  The plate is undamped and free-floating, so a
    per-step bias of the conserved moments (rounded equilibrium weights) would
    compound over the run; the kernel's collision keeps them exact."""
    p = configs.edge_crack_plate()
    s = slbm.Solver(p, "fp32")
    s.set_launch(6, 58)                   # the configuration the benchmark times
    s.step(p.steps)
    s.sync()
    u = s.displacement()
    sig = s.moments()[3]
    ref = Oracle(p)
    ref.step(p.steps)
    u_ref = ref.displacement()
    sig_ref = ref.moments()[3]
    raw = rel_l2(u, u_ref)
    d = u - u_ref
    deform = float(np.linalg.norm(d - rigid_part(d, p.mask)) / np.linalg.norm(u_ref))
    es = rel_l2(sig, sig_ref)
    print(f"crack1024x512 fp32 {p.steps} steps: rel L2 u = {raw:.3e}, without rigid-body part "
          f"{deform:.3e}, stress {es:.3e}")
    assert raw <= FP32_TOL
    assert es <= FP32_TOL


@pytest.mark.slow
@pytest.mark.parametrize("lam,tau,steps", [(0.1, 0.6, 50), (0.05, 0.55, 300)])
def test_hole_config_full_size(slbm, lam, tau, steps):
    """2048 x 2048 plate with the curved hole at full size in the
    configuration the benchmark's autotuner picks (two steps per launch, 10
    rows, XCD groups of 8).  lambda/mu = 2 (the workload's value) grows a boundary mode
    that swamps the solution within ~150 steps, so it is compared over the
    first 50; lambda/mu = 1 over 300."""
    p = configs.hole_plate(lam=lam, tau=tau)
    s = slbm.Solver(p, "fp32")
    s.set_launch(10, 58)
    s.set_xcd_group(8)
    s.step(steps)
    s.sync()
    ref = Oracle(p)
    ref.step(steps)
    e = rel_l2(s.displacement(), ref.displacement())
    print(f"hole2048 lam/mu={lam / 0.05:g} fp32 {steps} steps: rel L2 u = {e:.3e}")
    assert e <= FP32_TOL


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_moving_hole_plate_full_size(slbm, prec):
    """The 2048 x 2048 periodic plate with a fixed and a moving curved
    Dirichlet hole (the benchmark's workload for eq:bbnoncon with j* != 0),
    at full size in the two-step shape with XCD groups, 120 steps into the
    wall's ramp: displacement and moments against the reference."""
    p = configs.moving_hole_plate(steps=120, ramp_steps=60)
    s = slbm.Solver(p, prec)
    s.set_launch(10, 58)
    s.set_xcd_group(8)
    s.step(p.steps)
    s.sync()
    ref = Oracle(p, extended=(prec == "fp64"))
    ref.step(p.steps)
    e = compare(s, ref, prec)
    print(f"movinghole2048 {prec} {p.steps} steps: rel L2 u = {e:.3e}")


@pytest.mark.slow
def test_square4096_full_size_in_the_bench_launch_shape(slbm):
    """The 4096 x 4096 clamped/pulled plate the benchmark times, at full size
    in the configuration the autotuner picks for it (two steps per launch,
    10 rows, XCD groups of 8), fp32, 120 steps: displacement and moments
    against the reference."""
    p = configs.square_clamped_pulled(4096, steps=120)
    s = slbm.Solver(p, "fp32")
    s.set_launch(10, 58)
    s.set_xcd_group(8)
    s.step(p.steps)
    s.sync()
    ref = Oracle(p)
    ref.step(p.steps)
    e = compare(s, ref, "fp32")
    print(f"square4096 fp32 {p.steps} steps (10 x 58): rel L2 u = {e:.3e}")


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_largest_grid(slbm, prec):
    """The largest grid the library accepts, 16384 x 16384 = 2^28 sites, in
    the two-steps-per-launch shape: left edge clamped, right edge pulled by a
    step traction, 10 steps.  A site's state after k steps depends only on
    sites within 2k columns (one for the pull, one for the density stencil,
    per step), so the right-most columns must equal those of a 64-column
    plate with the same edges run by the reference, and every site farther
    than 2k columns from the pulled edge must still be exactly at rest."""
    n, k, w = 16384, 10, 64
    full = configs.square_clamped_pulled(n, steps=k)
    assert full.nx * full.ny == 1 << 28
    s = slbm.Solver(full, prec)
    s.set_launch(10, 58)
    s.step(k)
    s.sync()
    u = s.displacement()
    s.close()
    print(f"largest grid {prec}: {k} steps on {n} x {n} done", flush=True)
    crop = G.build_plate(w, n, lam=full.lam, mu=full.mu, tau=full.tau,
                         walls=G.edge_walls(w, n, left=0, right=1, bottom=2, top=2), groups=full.groups,
                         neumann_order=full.neumann_order, name="crop")
    ref = Oracle(crop, extended=(prec == "fp64"))
    ref.step(k)
    u_ref = ref.displacement()
    m = w - 2 * k - 2                              # columns beyond the cropped plate's own left edge's reach
    a, b = u[:, :, n - m:], u_ref[:, :, w - m:]
    e = rel_l2(a, b)
    print(f"largest grid {prec}: right-most {m} columns vs reference rel L2 {e:.3e}", flush=True)
    assert np.abs(b).max() > 0
    assert e <= (FP64_TOL if prec == "fp64" else FP32_TOL), e
    assert not np.any(u[:, :, : n - 2 * k - 1])


@pytest.mark.slow
def test_crack_tip_sif_fp32_follows_freund_k0(slbm):
    """The fp32 HIP path reproduces Freund's K^0 growth on the 1024 x 512
    edge crack (within 5 %) and the reference's own fit (within 1e-3)."""
    from crack_sif import sif_series
    p = configs.edge_crack_plate(steps=400)
    s = slbm.Solver(p, "fp32")
    t1 = p.ny // 2
    ratio, lag = sif_series(s.step, lambda: s.moments()[3][1], p, 1e-3 * p.mu, t1)
    o = Oracle(p)
    r_ref, lag_ref = sif_series(o.step, lambda: o.moments()[3][1], p, 1e-3 * p.mu, t1)
    print(f"crack tip K: fp32 sqrt(t) coefficient / Freund = {ratio:.4f} (reference {r_ref:.4f}), "
          f"onset lag {lag:.1f} steps")
    assert abs(ratio - 1) < 0.05
    assert 0 <= lag <= 40
    assert abs(ratio - r_ref) < 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paper_crack_follows_freund_k1(slbm, prec):
    """The HIP path on the paper's crack (section 5.2) past the first
    scattered waves: its stress intensity factor at P_1, sampled every
    second step to 2.1 l_c/c_d, equals the reference's sample by sample (to
    the bound the moment fields are held to), keeps
    its ratio to Freund's K^1 over [1, 1.75] l_c/c_d within 2 %, and rises
    fastest at the Rayleigh arrival."""
    from crack_sif import paper_crack_k1_window
    p = configs.paper_center_crack()
    s = slbm.Solver(p, prec)
    tau, K, drift, t_steep, t_ray = paper_crack_k1_window(s.step, lambda: s.moments()[3][0], p)
    o = Oracle(p, extended=(prec == "fp64"))
    _, K_ref, _, _, _ = paper_crack_k1_window(o.step, lambda: o.moments()[3][0], p)
    e = np.abs(K - K_ref).max() / np.abs(K_ref).max()
    print(f"paper crack {prec}: K at P_1 vs reference {e:.3e}; K/K^1 drift {drift:.4f}; "
          f"steepest rise at {t_steep:.3f} l_c/c_d (Rayleigh arrival {t_ray:.3f})")
    assert e <= (4 * FP64_TOL if prec == "fp64" else 1e-3), e     # the bounds on moment fields
    assert drift < 0.02, drift
    assert abs(t_steep - t_ray) < 0.05, (t_steep, t_ray)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_leaves_the_state_untouched(slbm, prec):
    """slbm_autotune times trial steps on the live plate; the state, the step
    count and the results must be exactly as without it."""
    p = mixed_plate(200, 90, seed=17, order=1)
    a = slbm.Solver(p, prec)
    a.step(25)
    seg, strip, us = a.autotune()
    assert seg >= 2 and strip in (58, 62, 64) and us > 0
    assert a.launch() == (seg, strip, a.launch()[2]) and a.launch()[2] in (0, 8)
    assert a.time()[0] == 25
    a.step(25)
    b = slbm.Solver(p, prec)
    b.step(50)
    assert np.array_equal(a.displacement(), b.displacement())
    assert np.array_equal(a.moments()[2], b.moments()[2])
