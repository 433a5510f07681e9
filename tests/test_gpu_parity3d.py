"""Parity of the three-dimensional HIP step (include/slbm3.h) with the CPU
reference (oracle/slbm3d.py), element by element on the same seeded inputs:
fp64 within 1e-12 relative L2 (against the reference's extended-precision
form), fp32 (fp64 displacement) within 1e-4.  Boxes are ragged against the
kernels' 64-site row chunks."""
import numpy as np
import pytest

from oracle.slbm3d import Oracle3D
from slbm_workloads import box3d as B

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def S3():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_04088_amd import slbm3
    slbm3.lib()
    return slbm3


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def err(a, b, unit):
    """(relative L2 error, whether it is within the rounding floor): the
    floor, 1e-15 sqrt(N) lattice units of the quantity (`unit` converts one
    lattice unit to user units), covers fields that are zero in exact
    arithmetic, such as the displacement before the first step."""
    d = float(np.linalg.norm(a - b))
    return d / max(float(np.linalg.norm(b)), 1e-300), d <= 1e-15 * np.sqrt(a.size) * unit


def units(box):
    """User units of one lattice unit: velocity, stress."""
    return np.sqrt(3 * box.mu / box.rho), 3 * box.mu


def run_both(S3, box, prec, steps, fields=None):
    s = S3.Solver3(box, prec)
    # fp64 parity at 1e-12 needs the reference's extended form: in float64 it
    # rounds its unshifted populations at about that level itself
    o = Oracle3D(box, extended=(prec == "fp64"))
    if fields is not None:
        s.init_fields(**fields)
        o.init_fields(**fields)
    s.step(steps)
    o.step(steps)
    s.sync()
    out = (s.displacement(), s.moments())
    ref = (o.displacement(), o.moments())
    st, t = s.time()
    assert st == steps
    s.close()
    return out, ref


def check(out, ref, tol, what, box):
    """Relative L2 of the displacement (cells), rho, j, P and sigma, each
    with its rounding floor."""
    (u, (rho, j, P, sig)), (ur, (rr, jr, Pr, sr)) = out, ref
    sv, ss = units(box)
    errs = {"u": err(u, ur, 1.0), "rho": err(rho, rr, box.rho),
            "j": err(j, jr, box.rho * sv), "P": err(P, Pr, ss), "sigma": err(sig, sr, ss)}
    print(what, {k: f"{v[0]:.2e}" + (" (floor)" if v[1] else "") for k, v in errs.items()})
    for k, (v, small) in errs.items():
        assert v <= tol or small, (what, k, v)


@pytest.mark.parametrize("prec,tol,steps", [("fp64", FP64_TOL, 30), ("fp32", FP32_TOL, 200)])
def test_periodic_box(S3, prec, tol, steps):
    box = B.periodic_box3(40, 12, 10, lam=0.08, mu=0.05, tau=0.6, force=(1e-6, -2e-6, 0.5e-6))
    fields = dict(vel=B.random_velocity(box, 21, 1e-3))
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"periodic {prec}", box)


@pytest.mark.parametrize("prec,tol,steps", [("fp64", FP64_TOL, 40), ("fp32", FP32_TOL, 300)])
def test_slab_with_both_wall_kinds(S3, prec, tol, steps):
    box = B.slab3(70, 6, 5, B.Wall3(B.DIRICHLET, (2e-4, -1e-4, 3e-4)), B.Wall3(B.NEUMANN, (1e-4, 2e-5, -3e-5)),
                  lam=0.05, mu=0.05, tau=0.55)
    fields = dict(vel=B.random_velocity(box, 22, 5e-4))
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"slab {prec}", box)


@pytest.mark.parametrize("prec,tol,steps", [("fp64", FP64_TOL, 40), ("fp32", FP32_TOL, 300)])
@pytest.mark.parametrize("qs,order", [((0.2, 0.8), 0), ((0.8, 0.3), 1), ((1.0, 0.15), 1)])
def test_slab_with_walls_off_the_lattice(S3, prec, tol, steps, qs, order):
    """Walls crossing the cut links at q != 1/2 (eq:bbnoncon, eq:abbnoncon),
    with rho_bd and the tangential stress at the boundary site or
    extrapolated along the link, both wall kinds on either side."""
    left, right = (B.Wall3(B.DIRICHLET, (2e-4, -1e-4, 3e-4), q=qs[0]),
                   B.Wall3(B.NEUMANN, (1e-4, 2e-5, -3e-5), q=qs[1]))
    if order == 1 and qs[0] > 0.9:
        left, right = (B.Wall3(B.NEUMANN, (-1e-4, 3e-5, 1e-5), q=qs[0]),
                       B.Wall3(B.DIRICHLET, (-1e-4, 2e-4, 0.0), q=qs[1]))
    box = B.slab3(70, 6, 5, left, right, lam=0.05, mu=0.05, tau=0.55, neumann_order=order)
    fields = dict(vel=B.random_velocity(box, 24, 5e-4))
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"slab q={qs} order {order} {prec}", box)


def test_single_site_thick_slab_off_the_lattice(S3):
    """nx = 1 with walls at q != 1/2: no site behind, so the rules take
    kappa = 0 and beta = 1 (and no extrapolation) as in the reference."""
    box = B.slab3(1, 7, 9, B.Wall3(B.NEUMANN, (1e-4, 0.0, 2e-5), q=0.3), B.Wall3(B.DIRICHLET, (-2e-4, 1e-5, 0.0), q=0.9),
                  lam=0.05, mu=0.05, tau=0.6, neumann_order=1)
    fields = dict(vel=B.random_velocity(box, 25, 1e-4))
    out, ref = run_both(S3, box, "fp64", 25, fields)
    check(out, ref, FP64_TOL, "nx=1 off the lattice", box)


@pytest.mark.parametrize("kinds", [(B.NEUMANN, B.NEUMANN), (B.DIRICHLET, B.DIRICHLET), (B.NEUMANN, B.DIRICHLET)])
def test_single_site_thick_slab(S3, kinds):
    """nx = 1: both walls act on the same sites."""
    box = B.slab3(1, 7, 9, B.Wall3(kinds[0], (1e-4, 0.0, 2e-5)), B.Wall3(kinds[1], (-2e-4, 1e-5, 0.0)),
                  lam=0.05, mu=0.05, tau=0.6)
    fields = dict(vel=B.random_velocity(box, 23, 1e-4))
    out, ref = run_both(S3, box, "fp64", 25, fields)
    check(out, ref, FP64_TOL, f"nx=1 {kinds}", box)


def test_initial_fields_all_given(S3):
    box = B.slab3(66, 5, 4, B.Wall3(B.NEUMANN), B.Wall3(B.DIRICHLET), lam=0.1, mu=0.05, tau=0.6)
    rng = np.random.default_rng(24)
    shape = (box.nz, box.ny, box.nx)
    fields = dict(rho=1.0 + 1e-4 * rng.standard_normal(shape), vel=B.random_velocity(box, 25, 2e-4),
                  sigma=1e-5 * rng.standard_normal((6,) + shape), u=1e-3 * rng.standard_normal((3,) + shape))
    for steps in (0, 7):
        out, ref = run_both(S3, box, "fp64", steps, fields)
        check(out, ref, FP64_TOL, f"init fields, {steps} steps", box)


def test_rest_stays_at_rest(S3):
    box = B.slab3(9, 3, 3, B.Wall3(B.DIRICHLET), B.Wall3(B.NEUMANN))
    for prec in ("fp32", "fp64"):
        s = S3.Solver3(box, prec)
        s.step(10)
        s.sync()
        assert np.abs(s.displacement()).max() == 0.0
        assert np.abs(s.moments()[1]).max() == 0.0
        s.close()


def test_non_finite_state_is_reported(S3):
    from paper_2208_04088_amd import slbm
    box = B.periodic_box3(8, 4, 4)
    s = S3.Solver3(box, "fp32")
    v = np.zeros((3,) + (box.nz, box.ny, box.nx))
    v[0, 1, 2, 3] = np.inf
    s.init_fields(vel=v)
    s.step(3)
    with pytest.raises(slbm.SlbmError) as e:
        s.sync()
    assert e.value.code == -4
    s.close()


@pytest.mark.slow
def test_cube128_fp32_against_the_reference(S3):
    """The benchmark's kind of box at 128^3: pulled slab, fp32, 20 steps from
    a random velocity field, every site against the reference."""
    box = B.cube_pulled(128, steps=20)
    fields = dict(vel=B.random_velocity(box, 26, 1e-4, smooth=3))
    out, ref = run_both(S3, box, "fp32", 20, fields)
    check(out, ref, FP32_TOL, "cube128 fp32", box)


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["periodic", "slab"])
def test_fp32_long_run(S3, kind):
    """5000 fp32 steps of an undamped periodic box, and of a slab with both
    wall kinds (its Dirichlet wall moves): the collision keeps the conserved
    moments free of the per-step bias of rounded weights, so the displacement
    error stays at rounding level rather than growing with the step count.
    (The reference's per-step cost on boxes this small makes 10^4 steps take
    minutes; the two-dimensional crack plate is checked over 10^4 steps.)"""
    if kind == "periodic":
        box = B.periodic_box3(48, 16, 16, lam=0.05, mu=0.05, tau=0.55)
        fields = dict(vel=B.random_velocity(box, 40, 1e-3))
    else:
        box = B.slab3(40, 8, 8, B.Wall3(B.DIRICHLET, (1e-4, 0.0, 0.0)), B.Wall3(B.NEUMANN, (5e-5, 1e-5, 0.0)))
        fields = None
    out, ref = run_both(S3, box, "fp32", 5000, fields)
    check(out, ref, FP32_TOL, f"{kind} fp32 5000 steps", box)


@pytest.mark.slow
def test_largest_box(S3):
    """The largest box the library accepts, 1024 x 1024 x 512 = 2^29 sites,
    fp32: clamped at x = -1/2, pulled at x = nx - 1/2 by a step traction,
    periodic in y and z.  The solution depends on x alone, so after 10 steps
    sampled (y, z) columns equal the first one bit for bit, and that column
    matches the reference run on a 1024 x 2 x 2 slab of the same walls."""
    nx, ny, nz, k = 1024, 1024, 512, 10
    walls = (B.Wall3(B.DIRICHLET), B.Wall3(B.NEUMANN, (5e-5, 0.0, 0.0)))
    box = B.slab3(nx, ny, nz, *walls)
    assert box.nx * box.ny * box.nz == 1 << 29
    s = S3.Solver3(box, "fp32")
    s.step(k)
    s.sync()
    u = s.displacement().reshape(3, ny * nz, nx)
    s.close()
    print(f"largest box: {k} steps on {nx} x {ny} x {nz} done", flush=True)
    cols = np.random.default_rng(5).integers(0, ny * nz, 4096)
    assert np.array_equal(u[:, cols, :], np.broadcast_to(u[:, :1, :], (3, cols.size, nx)))
    assert np.array_equal(u[:, -1, :], u[:, 0, :])
    o = Oracle3D(B.slab3(nx, 2, 2, *walls))
    o.step(k)
    u_ref = o.displacement()[:, 0, 0, :]
    e = rel_l2(u[:, 0, :], u_ref)
    print(f"largest box: x-profile vs reference rel L2 {e:.3e}", flush=True)
    assert np.abs(u_ref).max() > 0
    assert e <= FP32_TOL, e


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_device_outputs_match_host_outputs(S3, prec):
    """slbm3_displacement_device and slbm3_moments_device write what the host
    readouts return: the same doubles, or those doubles rounded to float."""
    import torch
    box = B.slab3(70, 5, 4, B.Wall3(B.DIRICHLET, (1e-4, 0.0, 0.0)), B.Wall3(B.NEUMANN, (5e-5, 1e-5, 0.0)))
    stream = torch.cuda.Stream()
    s = S3.Solver3(box, prec, stream=stream.cuda_stream)
    s.step(25)
    u_ref = s.displacement()
    ref = s.moments()
    with torch.cuda.stream(stream):
        u = torch.full((3, box.nz, box.ny, box.nx), 7.0, dtype=torch.float64, device="cuda")
    s.displacement_device(u.data_ptr())
    stream.synchronize()
    assert np.array_equal(u.cpu().numpy(), u_ref)
    for dt, tdt in (("fp64", torch.float64), ("fp32", torch.float32)):
        with torch.cuda.stream(stream):
            t = [torch.full(r.shape, 7.0, dtype=tdt, device="cuda") for r in ref]
        s.moments_device(*[x.data_ptr() for x in t], dtype=dt)
        stream.synchronize()
        for got, want in zip(t, ref):
            w = want.astype(np.float32) if dt == "fp32" else want
            assert np.array_equal(got.cpu().numpy(), w)
    s.close()


# ------------------------------------------------------------ cut links
def _thin_links(box):
    """Cut links whose opposite link at the same site is cut too."""
    cut = {(int(s), int(d)) for s, d in zip(box.links["site"], box.links["dir"])}
    return sum((s, d + 1 if d % 2 else d - 1) in cut for s, d in cut)


def _cavities(order, pressure=2e-4):
    """A box ragged against the 64-site rows (70 x 14 x 12) with two spherical
    cavities one site apart along x (the site between them has both x links
    cut: no site behind), one pressurised with a shear traction (Neumann),
    one a moving wall (Dirichlet), a body force.  lambda = mu and tau_bar =
    0.7: the rules' interpolation at small q (links that barely leave the
    material) stays stable there, so that a few hundred steps remain a
    meaningful fp32 comparison (the extrapolated Neumann form, order 1, grows
    a boundary mode even so and runs fewer steps)."""
    groups = [B.BCGroup3(B.NEUMANN, (2e-5, -1e-5, 3e-5), pressure), B.BCGroup3(B.DIRICHLET, (2e-4, -1e-4, 5e-5))]
    sph = [B.Sphere3(30.0, 6.6, 5.9, 3.0, 0), B.Sphere3(36.9, 7.1, 6.2, 3.0, 1)]
    return B.sphere_box3(70, 14, 12, sph, groups, lam=0.05, mu=0.05, tau=0.7, force=(2e-6, 0.0, -1e-6),
                         neumann_order=order)


@pytest.mark.parametrize("prec,tol,order,steps", [("fp64", FP64_TOL, 0, 40), ("fp64", FP64_TOL, 1, 40),
                                                  ("fp32", FP32_TOL, 0, 300), ("fp32", FP32_TOL, 1, 60)])
def test_cavities_with_cut_links(S3, prec, tol, order, steps):
    box = _cavities(order)
    assert _thin_links(box) > 0 and len(set(np.round(box.links["q"], 6))) > 20
    fields = dict(vel=B.random_velocity(box, 31 + order, 1e-3))
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"cavities {prec} order {order}", box)
    # void sites report zeros
    mk = ~box.mask.astype(bool)
    assert np.all(out[0][:, mk] == 0) and np.all(out[1][0][mk] == 0) and np.all(out[1][3][:, mk] == 0)


def test_pressurised_cavity_holds_its_hydrostatic_state(S3):
    """The oracle's patch test on the GPU: under the uniform stress -p I a
    cavity loaded by the pressure p stays at rest (fp64, 30 steps)."""
    p = 2e-4
    box = B.sphere_box3(70, 15, 14, [B.Sphere3(40.3, 6.8, 6.6, 3.7, 0)], [B.BCGroup3(B.NEUMANN, pressure=p)],
                        lam=0.1, mu=0.05, tau=0.6, neumann_order=1)
    sig = np.zeros((6, box.nz, box.ny, box.nx))
    sig[:3] = -p
    rho0 = np.full((box.nz, box.ny, box.nx), 1.0 + 3e-4)     # the lambda - mu terms act on drho
    with S3.Solver3(box, "fp64") as s:
        s.init_fields(rho=rho0, sigma=sig)
        s.step(12)
        s.sync()
        rho, j, P, sg = s.moments()
    mk = box.mask.astype(bool)
    assert np.abs(sg[:, mk] - sig[:, mk]).max() < 1e-12 * p / 1e-4
    assert np.abs(j[:, mk]).max() < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mask_without_void_matches_the_periodic_box(S3, prec):
    """A material mask with no void and no links runs the cut-link kernels
    on a box without boundaries: the same state as the periodic box, to the
    bit."""
    box = B.periodic_box3(70, 9, 7, lam=0.08, mu=0.05, tau=0.6, force=(1e-6, -2e-6, 0.5e-6))
    fields = dict(vel=B.random_velocity(box, 41, 1e-3))
    geo = B.Box3(**{**box.__dict__, "mask": np.ones((box.nz, box.ny, box.nx), np.uint8),
                    "links": np.zeros(0, B.LINK3_DTYPE), "groups": []})
    res = []
    for b in (box, geo):
        with S3.Solver3(b, prec) as s:
            s.init_fields(**fields)
            s.step(25)
            s.sync()
            res.append((s.displacement(), s.moments()))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        np.testing.assert_array_equal(a, b)


def _crack_links(box):
    """Cut links whose far end is material (a crack's faces)."""
    z, r = np.divmod(box.links["site"].astype(np.int64), box.ny * box.nx)
    y, x = np.divmod(r, box.nx)
    c = B.C3[box.links["dir"]]
    far = box.mask[(z + c[:, 2]) % box.nz, (y + c[:, 1]) % box.ny, (x + c[:, 0]) % box.nx]
    return int(far.sum())


def _cracked(order):
    """A ragged box (70 x 13 x 11) with a spherical cavity (Dirichlet, moving)
    and a penny-shaped crack of zero thickness (faces: traction-free below,
    a shear traction and pressure above), lambda = mu, tau_bar = 0.7."""
    groups = [B.BCGroup3(B.DIRICHLET, (2e-4, -1e-4, 5e-5)), B.BCGroup3(B.NEUMANN),
              B.BCGroup3(B.NEUMANN, (2e-5, -1e-5, 0.0), 1e-4)]
    return B.sphere_box3(70, 13, 11, [B.Sphere3(18.2, 6.4, 5.3, 3.2, 0)], groups, lam=0.05, mu=0.05, tau=0.7,
                         force=(0.0, 1e-6, -1e-6), neumann_order=order,
                         cracks=[B.PennyCrack3(45.3, 6.1, 5.4, 4.6, 1, 2)])


@pytest.mark.parametrize("prec,tol,order,steps", [("fp64", FP64_TOL, 0, 40), ("fp64", FP64_TOL, 1, 40),
                                                  ("fp32", FP32_TOL, 0, 300), ("fp32", FP32_TOL, 1, 60)])
def test_cavity_and_crack(S3, prec, tol, order, steps):
    box = _cracked(order)
    assert _crack_links(box) > 100
    assert _crack_links(box) < len(box.links)         # the cavity's links as well
    fields = dict(vel=B.random_velocity(box, 51 + order, 1e-3))
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"cavity and crack {prec} order {order}", box)


def test_penny_crack_leaves_an_in_plane_stress_alone_on_the_gpu(S3):
    """The oracle's crack patch test on the GPU (fp64, 30 steps): traction-free
    faces under a uniform stress in the crack's plane keep it exactly."""
    box = B.sphere_box3(70, 13, 10, [], [B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN)], lam=0.1, mu=0.05, tau=0.6,
                        neumann_order=1, cracks=[B.PennyCrack3(40.6, 6.2, 4.3, 4.1, 0, 1)])
    sig = np.zeros((6, box.nz, box.ny, box.nx))
    sig[0], sig[1], sig[3] = 3e-4, -1e-4, 2e-4
    with S3.Solver3(box, "fp64") as s:
        s.init_fields(sigma=sig)
        s.step(30)
        s.sync()
        rho, j, P, sg = s.moments()
    assert np.abs(sg - sig).max() < 1e-12
    assert np.abs(j).max() < 1e-13


@pytest.mark.slow
def test_cavities256_holds_its_hydrostatic_state(S3):
    """The benchmark's porous solid at full size, in its precision and launch
    configuration (256^3, 64 cavities, 1.7 M cut links, fp32): under the
    uniform stress -p I, with p the pressure on every cavity wall, the state
    is exact at any size (the oracle's patch test), so after 100 steps sigma
    is still -p I at every material site to fp32 rounding and j is 0; a wrong
    q, normal, group or record would disturb it by the order of p."""
    import torch
    box = B.cavities_box3(256)
    p = box.groups[0].pressure
    n = box.n_sites
    sig = np.zeros((6, n))
    sig[:3] = -p
    with S3.Solver3(box, "fp32") as s:
        s.init_fields(sigma=sig.reshape(6, box.nz, box.ny, box.nx))
        s.step(100)
        s.sync()
        dev = torch.device("cuda:0")
        sg = torch.empty((6, n), dtype=torch.float64, device=dev)
        j = torch.empty((3, n), dtype=torch.float64, device=dev)
        s.moments_device(j=j.data_ptr(), sigma=sg.data_ptr())
        torch.cuda.synchronize()
    mk = torch.from_numpy(box.mask.ravel().astype(bool)).to(dev)
    target = torch.tensor([-p, -p, -p, 0.0, 0.0, 0.0], dtype=torch.float64, device=dev)[:, None]
    err_s = float((sg - target)[:, mk].abs().max())
    err_j = float(j[:, mk].abs().max())
    print(f"cavities256 hydrostatic: max |sigma + p I| = {err_s:.3e} (p = {p:.1e}), max |j| = {err_j:.3e}", flush=True)
    assert err_s < 1e-4 * p and err_j < 1e-4 * p


def islands_box(n, sites, groups, pick, q=0.5, order=0, nx=None):
    """Islands of material in a periodic void (sites: (x, y, z)) of an
    nx x n x n box; every link from an island site into the void is cut at q,
    with the link's own direction as the outward normal and group pick(k)
    for direction k.  An isolated site has all 18 links cut, each thin."""
    nx = nx or n
    mask = np.zeros((n, n, nx), np.uint8)
    for x, y, z in sites:
        mask[z, y, x] = 1
    recs = []
    for x, y, z in sites:
        for k in range(1, 19):
            c = B.C3[k]
            if mask[(z + c[2]) % n, (y + c[1]) % n, (x + c[0]) % nx]:
                continue
            recs.append(((z * n + y) * nx + x, k, q, pick(k), tuple(c / np.linalg.norm(c)), -1, (0.0, 0.0, 0.0)))
    links = np.array(recs, dtype=B.LINK3_DTYPE).reshape(-1)
    return B.Box3(nx, n, n, lam=0.05, mu=0.05, tau=0.55, mask=mask, links=links, groups=list(groups),
                  name=f"islands{nx}x{n}x{n}", neumann_order=order)


# an isolated site, a pair, a face-diagonal pair, an L and a 2 x 2 x 2 block
ISLANDS3 = [(1, 1, 1), (4, 1, 1), (5, 1, 1), (1, 4, 4), (2, 5, 4), (1, 5, 1), (2, 5, 1), (1, 6, 1)] + \
           [(x, y, z) for x in (4, 5) for y in (4, 5) for z in (4, 5)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_box_without_material(S3, prec):
    """An empty box (every site void, no links) steps and reads out zeros,
    as the reference does."""
    box = islands_box(9, [], [B.BCGroup3(B.NEUMANN)], lambda k: 0, nx=70)
    assert box.n_material == 0 and len(box.links) == 0
    out, ref = run_both(S3, box, prec, 20)
    assert not np.any(out[0]) and not any(np.any(m) for m in out[1])
    check(out, ref, FP64_TOL if prec == "fp64" else FP32_TOL, f"empty box {prec}", box)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("q", [0.5, 0.3])
def test_islands_with_moving_walls(S3, prec, tol, q):
    """Islands of one to eight sites, an isolated site among them, carried by
    moving Dirichlet walls on every link (thin links throughout), 40 steps."""
    box = islands_box(8, ISLANDS3, [B.BCGroup3(B.DIRICHLET, (1e-4, -2e-4, 3e-4))], lambda k: 0, q=q)
    out, ref = run_both(S3, box, prec, 40)
    check(out, ref, tol, f"islands {prec} q {q}", box)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("order", [0, 1])
def test_loaded_islands_few_steps(S3, prec, tol, order):
    """Islands with clamped links facing +x and Neumann links under a
    traction and a pressure elsewhere.  Free islands are violently unstable
    under the Neumann rule (rounding noise grows about threefold per step),
    so the comparison stops after 5 steps, while the state is still small."""
    groups = [B.BCGroup3(B.DIRICHLET), B.BCGroup3(B.NEUMANN, (3e-5, 1e-5, 0.0), 1e-5)]
    box = islands_box(8, ISLANDS3, groups, lambda k: 0 if B.C3[k][0] > 0 else 1, q=0.4, order=order)
    out, ref = run_both(S3, box, prec, 5)
    check(out, ref, tol, f"loaded islands {prec} order {order}", box)


def random_groups(rng, count):
    """Boundary groups of either kind with small seeded values (user units),
    a pressure on some Neumann groups, a ramp on some groups."""
    groups = []
    for _ in range(count):
        kind = int(rng.choice([B.DIRICHLET, B.NEUMANN]))
        value = tuple(float(v) for v in rng.uniform(-5e-5, 5e-5, 3))
        pressure = float(rng.uniform(0.0, 2e-4)) if kind == B.NEUMANN and rng.random() < 0.5 else 0.0
        ramp = rng.random() < 0.3
        groups.append(B.BCGroup3(kind, value, pressure, profile=B.RAMP if ramp else B.STEP,
                                 ramp_time=float(rng.uniform(3.0, 20.0)) if ramp else 0.0))
    return groups


def random_box(rng, block):
    """A seeded general geometry: one to three spherical cavities and up to
    two penny cracks in a box ragged against the 64-site rows, or (block) a
    rectangular block with a group per face (edges of both kinds, where the
    two faces share a profile); lambda/mu in [0.5, 1], tau_bar in
    [0.55, 0.8], a body force, either Neumann order."""
    nx, ny, nz = int(rng.integers(14, 90)), int(rng.integers(10, 17)), int(rng.integers(10, 15))
    lm, mu = float(rng.uniform(0.5, 1.0)), 0.05
    common = dict(lam=lm * mu, mu=mu, tau=float(rng.uniform(0.55, 0.8)),
                  force=tuple(float(v) for v in rng.uniform(-2e-6, 2e-6, 3)), neumann_order=int(rng.integers(2)))
    if block:
        groups = random_groups(rng, 6)
        for g in groups:                     # faces meeting at an edge share one profile
            g.profile, g.ramp_time = B.STEP, 0.0
        lo = [int(rng.integers(1, 4)) for _ in range(3)]
        hi = [int(rng.integers(l + 1, n - 1)) for l, n in zip(lo, (nx, ny, nz))]
        return B.block_box3(nx, ny, nz, lo, hi, list(range(6)), groups, **common)
    groups = random_groups(rng, int(rng.integers(1, 5)))
    sph = []
    for _ in range(int(rng.integers(1, 4))):
        R = float(rng.uniform(1.2, min(ny, nz) / 3.2))
        c = [float(rng.uniform(R + 1, n - R - 2)) for n in (nx, ny, nz)]
        sph.append(B.Sphere3(*c, R, int(rng.integers(len(groups)))))
    cracks = []
    for _ in range(int(rng.integers(0, 3))):
        R = float(rng.uniform(1.5, min(ny, nz) / 3.0))
        cx, cy = float(rng.uniform(R + 1, nx - R - 2)), float(rng.uniform(R + 1, ny - R - 2))
        cracks.append(B.PennyCrack3(cx, cy, int(rng.integers(2, nz - 2)) + 0.5, R,
                                    int(rng.integers(len(groups))), int(rng.integers(len(groups)))))
    return B.sphere_box3(nx, ny, nz, sph, groups, cracks=cracks, **common)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_random_geometries(S3, prec, tol):
    """Twelve seeded geometries (cavities, cracks, blocks; groups of both
    kinds, pressures, ramps, either Neumann order) from a seeded velocity
    field, 12 steps each, against the reference."""
    rng = np.random.default_rng(2208)
    for i in range(12):
        box = random_box(rng, block=(i % 3 == 2))
        fields = dict(vel=B.random_velocity(box, 500 + i, 1e-4))
        print(f"random geometry {i}: {box.nx}x{box.ny}x{box.nz}, {len(box.links)} links, "
              f"{int((box.links['group2'] >= 0).sum())} on edges, order {box.neumann_order}", flush=True)
        out, ref = run_both(S3, box, prec, 12, fields)
        check(out, ref, tol, f"random geometry {i} {prec}", box)


@pytest.mark.parametrize("prec,tol,steps", [("fp64", FP64_TOL, 30), ("fp32", FP32_TOL, 200)])
def test_narrow_box_with_cut_links(S3, prec, tol, steps):
    """A box narrower than one 64-site chunk (30 x 15 x 13: each workgroup of
    the step takes four rows, across z planes too, and the last one is
    partial) with a cavity and a crack: the workgroups' record ranges and the
    staging of their sites' populations."""
    groups = [B.BCGroup3(B.NEUMANN, (0.0, 0.0, 0.0), 1e-4), B.BCGroup3(B.DIRICHLET, (1e-4, 0.0, -2e-4)),
              B.BCGroup3(B.NEUMANN)]
    box = B.sphere_box3(30, 15, 13, [B.Sphere3(9.3, 7.2, 6.1, 3.4, 0)], groups, lam=0.05, mu=0.05, tau=0.7,
                        neumann_order=0, cracks=[B.PennyCrack3(21.4, 7.6, 6.5, 4.2, 1, 2)])
    assert ((box.nx + 63) // 64 * box.ny * box.nz) % 4 != 0 and _crack_links(box) > 50
    fields = dict(vel=B.random_velocity(box, 61, 1e-3))
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"narrow box {prec}", box)


def _block(order):
    """A 64 x 9 x 8 block in a 70 x 13 x 12 box (ragged rows, a partial last
    workgroup), one group per face: clamped and moving Dirichlet faces,
    loaded and free Neumann faces; its edges carry two faces' groups."""
    groups = [B.BCGroup3(B.DIRICHLET, (2e-4, 0.0, 0.0)), B.BCGroup3(B.NEUMANN, (3e-5, 0.0, 0.0)),
              B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN, (0.0, 1e-5, 2e-5), 5e-5),
              B.BCGroup3(B.NEUMANN), B.BCGroup3(B.DIRICHLET)]
    return B.block_box3(70, 13, 12, (3, 2, 2), (66, 10, 9), list(range(6)), groups, lam=0.05, mu=0.05, tau=0.7,
                        force=(0.0, 1e-6, 0.0), neumann_order=order)


@pytest.mark.parametrize("prec,tol,order,steps", [("fp64", FP64_TOL, 0, 40), ("fp64", FP64_TOL, 1, 40),
                                                  ("fp32", FP32_TOL, 0, 300), ("fp32", FP32_TOL, 1, 60)])
def test_block_with_edges(S3, prec, tol, order, steps):
    box = _block(order)
    assert (box.links["group2"] >= 0).sum() > 100
    fields = dict(vel=B.random_velocity(box, 71, 1e-3) * box.mask)
    out, ref = run_both(S3, box, prec, steps, fields)
    check(out, ref, tol, f"block {prec} order {order}", box)


def test_block_holds_a_uniform_stress_on_the_gpu(S3):
    """The oracle's block patch test on the GPU (fp64, order 1, 12 steps, at
    lambda/mu = 1.3 so that the lambda - mu terms of the edge rule count):
    faces and edges loaded by sigma.n keep the uniform stress sigma.  (The
    extrapolated rule's free-wall mode amplifies rounding quickly above
    lambda = mu, in the reference as here, hence the short run.)"""
    sig3 = np.array([[3e-4, 1e-4, -2e-4], [1e-4, -1e-4, 1.5e-4], [-2e-4, 1.5e-4, 2e-4]])
    faces = [(-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, -1.0), (0.0, 0.0, 1.0)]
    groups = [B.BCGroup3(B.NEUMANN, tuple(sig3 @ np.array(n))) for n in faces]
    box = B.block_box3(70, 13, 12, (3, 2, 2), (66, 10, 9), list(range(6)), groups, lam=0.065, mu=0.05, tau=0.6,
                       neumann_order=1)
    sig = np.zeros((6, box.nz, box.ny, box.nx))
    for k, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        sig[k] = sig3[i, j]
    with S3.Solver3(box, "fp64") as s:
        s.init_fields(sigma=sig)
        s.step(30)
        s.sync()
        rho, j, P, sg = s.moments()
    mk = box.mask.astype(bool)
    assert np.abs(sg[:, mk] - sig[:, mk]).max() < 1e-12
    assert np.abs(j[:, mk]).max() < 1e-13


@pytest.mark.parametrize("prec,tol,steps", [("fp64", FP64_TOL, 40), ("fp32", FP32_TOL, 300)])
@pytest.mark.parametrize("order", [0, 1])
def test_ramped_walls(S3, prec, tol, steps, order):
    """Wall planes off the lattice whose values ramp up over 25 and 60 steps
    (the wall values at the time of the state each rule reads)."""
    dt = np.sqrt(1.0 / (3 * 0.05))
    walls = (B.Wall3(B.DIRICHLET, (1e-4, -2e-4, 5e-5), q=0.3, profile=B.RAMP, ramp_time=25 * dt),
             B.Wall3(B.NEUMANN, (5e-5, 1e-5, -2e-5), q=0.8, profile=B.RAMP, ramp_time=60 * dt))
    box = B.slab3(70, 6, 5, *walls, lam=0.05, mu=0.05, tau=0.6, neumann_order=order)
    out, ref = run_both(S3, box, prec, steps if order == 0 else min(steps, 60))
    check(out, ref, tol, f"ramped walls {prec} order {order}", box)


@pytest.mark.parametrize("prec,tol,steps", [("fp64", FP64_TOL, 40), ("fp32", FP32_TOL, 300)])
def test_ramped_groups(S3, prec, tol, steps):
    """Cut links whose groups ramp over different times (a pressurised cavity,
    a moving cavity, a loaded crack face, a block's faces and edges sharing
    one ramp), from rest."""
    dt = np.sqrt(1.0 / (3 * 0.05))
    R = lambda T: dict(profile=B.RAMP, ramp_time=T * dt)
    groups = [B.BCGroup3(B.NEUMANN, (0.0, 0.0, 0.0), 2e-4, **R(30)), B.BCGroup3(B.DIRICHLET, (2e-4, -1e-4, 0.0), **R(12)),
              B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN, (3e-5, 0.0, 1e-5), **R(45))]
    box = B.sphere_box3(70, 14, 12, [B.Sphere3(14.2, 6.6, 5.9, 3.0, 0), B.Sphere3(30.4, 7.1, 6.2, 2.8, 1)], groups,
                        lam=0.05, mu=0.05, tau=0.7, cracks=[B.PennyCrack3(50.3, 6.8, 5.4, 4.1, 2, 3)])
    out, ref = run_both(S3, box, prec, steps)
    check(out, ref, tol, f"ramped groups {prec}", box)
    bgroups = [B.BCGroup3(B.NEUMANN, (2e-5, 0.0, 0.0), **R(20))] * 5 + [B.BCGroup3(B.NEUMANN, (0.0, 0.0, 1e-5), **R(20))]
    block = B.block_box3(70, 11, 10, (3, 2, 2), (66, 8, 7), list(range(6)), bgroups, lam=0.05, mu=0.05, tau=0.7)
    out, ref = run_both(S3, block, prec, steps)
    check(out, ref, tol, f"ramped block {prec}", block)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["slab", "geometry"])
def test_checkpoint_resume_is_bit_identical(S3, prec, kind):
    """slbm3_save after k steps, slbm3_load into a fresh handle of the same
    box, m more steps: the same state, to the bit, as k + m steps without
    interruption (ramped values, extrapolated rules and, with cut links, the
    rule values the next step reads are part of the state)."""
    dt = np.sqrt(1.0 / (3 * 0.05))
    if kind == "slab":
        box = B.slab3(70, 6, 5, B.Wall3(B.DIRICHLET, (1e-4, 0.0, 2e-5), q=0.3, profile=B.RAMP, ramp_time=20 * dt),
                      B.Wall3(B.NEUMANN, (5e-5, 1e-5, 0.0), q=0.7), lam=0.05, mu=0.05, tau=0.6, neumann_order=1)
    else:
        box = _block(1)
    k, m = 13, 11
    fields = dict(vel=B.random_velocity(box, 81, 1e-3) * (1 if box.mask is None else box.mask))
    with S3.Solver3(box, prec) as a:
        a.init_fields(**fields)
        a.step(k + m)
        a.sync()
        u_ref, mom_ref = a.displacement(), a.moments()
    with S3.Solver3(box, prec) as b:
        b.init_fields(**fields)
        b.step(k)
        b.sync()
        ck = b.save()
    with S3.Solver3(box, prec) as c:
        c.load(ck)
        assert c.time()[0] == k
        c.step(m)
        c.sync()
        u, mom = c.displacement(), c.moments()
    assert np.array_equal(u, u_ref)
    for x, y in zip(mom, mom_ref):
        assert np.array_equal(x, y)


def test_checkpoint_of_another_geometry_is_refused(S3):
    """A checkpoint loads only into a handle of the same geometry: a cavity
    moved by one site (same box, same number of cut links, so the state has
    the same size) and a slab whose wall sits at another q are refused."""
    from paper_2208_04088_amd import slbm
    groups = [B.BCGroup3(B.NEUMANN, (0.0, 0.0, 0.0), 1e-4)]
    a = B.sphere_box3(30, 14, 12, [B.Sphere3(10.3, 6.6, 5.8, 3.1, 0)], groups)
    b = B.sphere_box3(30, 14, 12, [B.Sphere3(11.3, 6.6, 5.8, 3.1, 0)], groups)
    assert len(a.links) == len(b.links) and not np.array_equal(a.mask, b.mask)
    s1 = B.slab3(20, 6, 5, B.Wall3(B.DIRICHLET), B.Wall3(B.NEUMANN, q=0.5))
    s2 = B.slab3(20, 6, 5, B.Wall3(B.DIRICHLET), B.Wall3(B.NEUMANN, q=0.3))
    for x, y in ((a, b), (s1, s2)):
        with S3.Solver3(x, "fp32") as s:
            s.step(3)
            ck = s.save()
        with S3.Solver3(y, "fp32") as t:
            with pytest.raises(slbm.SlbmError) as e:
                t.load(ck)
            assert e.value.code == -1 and "geometry" in str(e.value)
        with S3.Solver3(x, "fp32") as t:
            t.load(ck)
            assert t.time()[0] == 3
