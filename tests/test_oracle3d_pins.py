"""Pins of the three-dimensional (D3Q19) CPU reference against what the
mathematics fixes: lattice isotropy, the equilibrium's moments, conservation,
exact patch tests of both wall rules, axis symmetry, the wave speeds of
isotropic elasticity (sections 2-3, eq:navier), the one-dimensional step-load
amplitude, and a brute-force loop implementation on a tiny box."""
import itertools

import numpy as np
import pytest

from oracle.slbm3d import C, OPP, Q, W, Oracle3D, equilibrium, sym_to_full
from slbm_workloads import box3d as B
from tests.naive3d import naive_step


def test_lattice_isotropy():
    """D3Q19: weights sum to 1, odd moments vanish, second moment c_s^2 I,
    fourth moment c_s^4 (delta delta + delta delta + delta delta)."""
    d = np.eye(3)
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("i,ia->a", W, C), 0)
    assert np.allclose(np.einsum("i,ia,ib->ab", W, C, C), d / 3)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", W, C, C, C), 0)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-15)
    assert (C[OPP] == -C).all() and Q == 19


def test_equilibrium_has_the_given_moments():
    """eq:fieq: sum f_eq = rho, sum f_eq c = j, sum f_eq c c = P."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = rng.uniform(0.8, 1.2)
        j = rng.normal(size=3) * 0.1
        A = rng.normal(size=(3, 3)) * 0.1
        P = A + A.T
        f = equilibrium(np.array([rho]), j[:, None], P[:, :, None])[:, 0]
        assert f.sum() == pytest.approx(rho, abs=1e-14)
        assert np.allclose(C.T @ f, j, atol=1e-14)
        assert np.allclose(np.einsum("i,ia,ib->ab", f, C, C), P, atol=1e-14)


def test_rest_state_stays_at_rest_with_both_walls():
    b = B.slab3(7, 3, 4, B.Wall3(B.DIRICHLET), B.Wall3(B.NEUMANN), lam=0.1, mu=0.05, tau=0.6)
    o = Oracle3D(b)
    f0 = o.populations()
    o.step(6)
    assert np.abs(o.populations() - f0).max() < 1e-14
    assert np.abs(o.displacement()).max() < 1e-14


def test_mass_conserved_and_momentum_gains_the_body_force():
    """Periodic box: total mass is constant; with lambda = mu the density
    gradient term vanishes and total momentum grows by the body force per
    site per step (in user units, j gains rho F dt)."""
    b = B.periodic_box3(9, 7, 6, lam=0.05, mu=0.05, tau=0.55, force=(2e-5, -1e-5, 3e-5))
    o = Oracle3D(b)
    o.init_fields(vel=B.random_velocity(b, 11, 1e-3))
    r0, j0 = o.moments()[0].sum(), o.moments()[1].sum(axis=(1, 2, 3))
    steps = 12
    o.step(steps)
    r1, j1 = o.moments()[0].sum(), o.moments()[1].sum(axis=(1, 2, 3))
    assert abs(r1 - r0) < 1e-12 * r0
    dt = o.dt_user
    assert np.allclose(j1 - j0, np.array(b.force) * b.n_sites * steps * dt, rtol=1e-9, atol=1e-15)


def test_momentum_not_conserved_when_lambda_differs_from_mu():
    """The (mu - lambda)/rho grad(rho) source divides by the local density, so
    momentum is conserved exactly only at lambda = mu: the check above would
    not catch a dropped source term, this one does."""
    b = B.periodic_box3(9, 7, 6, lam=0.1, mu=0.05, tau=0.6)
    o = Oracle3D(b)
    o.init_fields(vel=B.random_velocity(b, 12, 1e-2))
    j0 = o.moments()[1].sum(axis=(1, 2, 3))
    o.step(8)
    j1 = o.moments()[1].sum(axis=(1, 2, 3))
    assert np.abs(j1 - j0).max() > 1e-12


def test_axis_permutation_symmetry():
    """Cyclic relabelling x -> y -> z -> x of the initial field relabels the
    solution the same way (the lattice is invariant under it)."""
    b = B.periodic_box3(6, 6, 6, lam=0.08, mu=0.05, tau=0.6)
    v = B.random_velocity(b, 5, 1e-3)
    o1 = Oracle3D(b)
    o1.init_fields(vel=v)
    o1.step(5)
    u1 = o1.displacement()
    # array axes are (z, y, x); the map (x, y, z) -> (y, z, x) sends component x to y
    vp = np.empty_like(v)
    vp[1], vp[2], vp[0] = (np.moveaxis(v[k], (0, 1, 2), (2, 0, 1)) for k in range(3))
    o2 = Oracle3D(b)
    o2.init_fields(vel=vp)
    o2.step(5)
    u2 = o2.displacement()
    for k, kp in ((0, 1), (1, 2), (2, 0)):
        assert np.allclose(np.moveaxis(u1[k], (0, 1, 2), (2, 0, 1)), u2[kp], atol=1e-16, rtol=1e-11)


@pytest.mark.parametrize("order", [0, 1])
def test_cavities_are_equivariant_under_axis_relabelling(order):
    """The cyclic relabelling x -> y -> z -> x of a box with cavities (one
    pressurised with a shear traction, one moving), of its groups' vectors and
    of the initial field relabels the solution: the per-link directions,
    normals, q and group values are handled alike along every axis (a
    transposed normal or traction component breaks it)."""
    n = 12
    groups = [B.BCGroup3(B.NEUMANN, (2e-4, -1e-4, 3e-4), 1e-4), B.BCGroup3(B.DIRICHLET, (1e-3, -2e-3, 5e-4))]
    sph = [(3.7, 4.4, 5.2, 2.3, 0), (8.1, 7.2, 6.3, 2.1, 1)]

    def rot(v):                      # (x, y, z) -> (z, x, y): component x goes to y
        return (v[2], v[0], v[1])

    def box(spheres, grps):
        return B.sphere_box3(n, n, n, [B.Sphere3(*c, R, g) for *c, R, g in spheres], grps, lam=0.08, mu=0.05,
                             tau=0.6, neumann_order=order)

    b1 = box(sph, groups)
    b2 = box([(*rot(c[:3]), c[3], c[4]) for c in sph],
             [B.BCGroup3(g.kind, rot(g.value), g.pressure) for g in groups])
    v = B.random_velocity(b1, 6, 1e-3)
    vp = np.empty_like(v)
    vp[1], vp[2], vp[0] = (np.moveaxis(v[k], (0, 1, 2), (2, 0, 1)) for k in range(3))
    o1, o2 = Oracle3D(b1), Oracle3D(b2)
    o1.init_fields(vel=v)
    o2.init_fields(vel=vp)
    o1.step(6)
    o2.step(6)
    u1, u2 = o1.displacement(), o2.displacement()
    assert np.abs(u1).max() > 1e-4
    for k, kp in ((0, 1), (1, 2), (2, 0)):
        assert np.allclose(np.moveaxis(u1[k], (0, 1, 2), (2, 0, 1)), u2[kp], atol=1e-15, rtol=1e-10)


def _mode_frequency(o, kvec, comp, steps):
    """Angular frequency (per step) of the standing mode sum_x j(x) sin(k.x)
    along `comp`: the slope of its zero-crossing times, each located by
    linear interpolation between steps (damping does not move them)."""
    nz, ny, nx = o.shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = np.sin(kvec[0] * xx + kvec[1] * yy + kvec[2] * zz)
    a = []
    for _ in range(steps):
        o.step(1)
        j = o.moments()[1]
        a.append(float((np.tensordot(comp, j, 1) * s).sum()))
    a = np.array(a)
    t = np.arange(1, steps + 1)
    zc = np.flatnonzero(np.sign(a[1:]) != np.sign(a[:-1]))
    tc = np.array([t[i] + a[i] / (a[i] - a[i + 1]) for i in zc])
    half = np.polyfit(np.arange(len(tc)), tc, 1)[0]
    return np.pi / half


@pytest.mark.parametrize("lam_over_mu", [1.0, 0.769, 2.0])
def test_wave_speeds_along_an_axis(lam_over_mu):
    """Shear waves travel at c_s = sqrt(mu/rho), pressure waves at
    c_d = sqrt((lambda + 2 mu)/rho) (eq:navier), here in lattice units
    (c_s^2 = 1/3, c_d^2 = lambda_L + 2/3), k = 2 pi/64."""
    n = 64
    tau = 0.6 if lam_over_mu > 1.5 else 0.55
    k = 2 * np.pi / n
    for comp, target in (((0.0, 1.0, 0.0), np.sqrt(1 / 3)), ((1.0, 0.0, 0.0), np.sqrt(lam_over_mu / 3 + 2 / 3))):
        b = B.periodic_box3(n, 1, 1, lam=0.05 * lam_over_mu, mu=0.05, tau=tau)
        o = Oracle3D(b)
        x = np.arange(n)
        v = np.zeros((3, 1, 1, n))
        v[int(np.argmax(comp))] = 1e-4 * np.sin(k * x)
        o.init_fields(vel=v)
        w = _mode_frequency(o, (k, 0, 0), np.array(comp), 300)
        assert w / k == pytest.approx(target, rel=3e-3), (comp, w / k, target)


def test_wave_speeds_along_a_face_diagonal():
    """The same speeds for k along (1, 1, 0): exercises the diagonal links
    and their weights."""
    n = 32
    kk = 2 * np.pi / n
    kvec = (kk, kk, 0.0)
    kn = np.sqrt(2) * kk
    b = B.periodic_box3(n, n, 1, lam=0.05, mu=0.05, tau=0.55)
    zz, yy, xx = np.meshgrid(np.arange(1), np.arange(n), np.arange(n), indexing="ij")
    s = np.sin(kk * xx + kk * yy)
    for comp, target in (((1 / np.sqrt(2), -1 / np.sqrt(2), 0.0), np.sqrt(1 / 3)),
                         ((1 / np.sqrt(2), 1 / np.sqrt(2), 0.0), np.sqrt(1.0))):
        o = Oracle3D(b)
        v = np.array(comp)[:, None, None, None] * 1e-4 * s[None]
        o.init_fields(vel=v)
        w = _mode_frequency(o, kvec, np.array(comp), 160)
        assert w / kn == pytest.approx(target, rel=5e-3), (comp, w / kn, target)


@pytest.mark.parametrize("q,order", [(0.5, 0), (0.2, 0), (0.8, 0), (0.5, 1), (0.3, 1), (1.0, 1)])
def test_neumann_walls_hold_a_uniform_stress(q, order):
    """Patch test of eq:abbcon (q = 1/2) and eq:abbnoncon: a uniform stress
    with the matching tractions on both walls (t* = sigma.n, n = -x and +x)
    is an exact steady state, for every component, at any q and with rho_bd
    and the tangential stress at the site or extrapolated: a wrong sign or
    projection in the boundary stress, a dropped tangential block, or kappa
    and beta that do not satisfy 1 + 2 kappa = 2 beta break it."""
    s0 = np.array([2e-4, -1e-4, 3e-4, 1.5e-4, -2.5e-4, 0.5e-4])   # xx yy zz xy xz yz
    S = sym_to_full(s0[:, None])[:, :, 0]
    left = B.Wall3(B.NEUMANN, tuple(-S[:, 0]), q=q)
    right = B.Wall3(B.NEUMANN, tuple(S[:, 0]), q=1.0 - q / 2)
    b = B.slab3(6, 3, 2, left, right, lam=0.1, mu=0.05, tau=0.6, neumann_order=order)
    o = Oracle3D(b)
    sig = np.broadcast_to(s0[:, None, None, None], (6,) + o.shape)
    o.init_fields(sigma=sig)
    m0 = o.moments()
    o.step(7)
    m1 = o.moments()
    # rounding leaves ~1e-15; a wrong rule errs by the order of the load (1e-4)
    assert np.abs(m1[3] - sig).max() < 1e-13
    assert np.abs(m1[1]).max() < 1e-13
    assert np.abs(m1[0] - m0[0]).max() < 1e-13


@pytest.mark.parametrize("q", [0.5, 0.2, 0.8, 1.0])
def test_dirichlet_walls_carry_a_uniform_translation(q):
    """Patch test of eq:bbcon (q = 1/2) and eq:bbnoncon: walls moving with the
    material's uniform velocity keep it in rigid translation at any q (the
    interpolation weights satisfy beta - kappa = 1); the displacement grows
    as v t."""
    v0 = np.array([3e-4, -2e-4, 1e-4])
    b = B.slab3(5, 2, 3, B.Wall3(B.DIRICHLET, tuple(v0), q=q), B.Wall3(B.DIRICHLET, tuple(v0), q=q),
                lam=0.1, mu=0.05, tau=0.6)
    o = Oracle3D(b)
    o.init_fields(vel=np.broadcast_to(v0[:, None, None, None], (3,) + o.shape))
    o.step(9)
    rho, j, P, sig = o.moments()
    # rounding leaves ~1e-16; a wrong rule errs by the order of v0 (1e-4)
    assert np.abs(j - v0[:, None, None, None]).max() < 1e-13
    assert np.abs(sig).max() < 1e-13
    u = o.displacement()
    assert np.abs(u - (v0 * 9 * o.dt_user)[:, None, None, None]).max() < 1e-13


@pytest.mark.parametrize("mode,q,order", [("tension", 0.5, 0), ("shear", 0.5, 0), ("tension", 0.2, 0),
                                          ("shear", 0.8, 0), ("tension", 0.3, 1), ("shear", 0.5, 1)])
def test_step_traction_launches_the_one_dimensional_wave(mode, q, order):
    """A step tension sigma_xx = s0 (or shear sigma_xy = s0) on the face of a
    long slab (the wall crossing the boundary links at q) sends a plane
    pressure (shear) wave in at c_d (c_s); behind its front the material moves
    with v = -s0/(rho c) along x (y), by momentum balance across the front,
    until the reflection from the free far face returns.  The shear case pins
    the tangential part of the Neumann rule's boundary stress; q != 1/2 and
    the extrapolated rule pin eq:abbnoncon's kappa, beta and rho_bd."""
    nx, s0 = 240, 1e-4
    mu, lam = 0.05, 0.05
    k = 0 if mode == "tension" else 1
    t = [0.0, 0.0, 0.0]
    t[k] = -s0
    b = B.slab3(nx, 1, 1, B.Wall3(B.NEUMANN, tuple(t), q=q), B.Wall3(B.NEUMANN, q=q), lam=lam, mu=mu,
                tau=0.55, neumann_order=order)
    o = Oracle3D(b)
    c_lat = np.sqrt(lam / mu / 3 + 2 / 3) if mode == "tension" else np.sqrt(1 / 3)
    steps = int(0.75 * nx / c_lat)
    o.step(steps)
    rho, j, P, sig = o.moments()
    v = j[k, 0, 0] / rho[0, 0, 0]
    c_user = np.sqrt((lam + 2 * mu) / b.rho) if mode == "tension" else np.sqrt(mu / b.rho)
    behind = v[20:int(0.5 * nx)]
    assert np.mean(behind) == pytest.approx(-s0 / (b.rho * c_user), rel=0.02)
    assert np.abs(v[int(0.9 * nx):]).max() < 1e-3 * s0 / (b.rho * c_user)
    other = j[1 - k, 0, 0] / rho[0, 0, 0]
    assert np.abs(other).max() < 1e-6 * s0 / (b.rho * c_user)


@pytest.mark.parametrize("kind", ["neumann", "dirichlet"])
@pytest.mark.parametrize("q_left,q_right", [(0.5, 0.5), (0.3, 0.8), (0.9, 0.15)])
def test_wall_rules_are_exact_for_linear_fields(kind, q_left, q_right):
    """Section 4.2 in three dimensions: for an equilibrium field varying
    linearly across the wall, a cut link returns the population the lattice
    would have streamed in from the virtual site x + c_i had the field
    continued -- for every q.  The Neumann rule (j = 0) needs rho_bd and the
    tangential block of the stress extrapolated along the link (order 1) and
    the traction of the field at the wall plane; the Dirichlet rule, a linear
    velocity field with the wall velocity at the wall plane.  Walls at
    x = -q_left and x = nx - 1 + q_right; lambda = mu, so the source term
    vanishes and the collision leaves the field as it is."""
    nx, ny, nz = 5, 3, 2
    mu = lam = 0.05

    def fields(x):          # lattice units: rho, j, P (full 3 x 3)
        if kind == "neumann":
            P6 = np.array([3e-4 - 1e-4 * x, 2e-4 + 5e-5 * x, -1e-4 + 2e-5 * x,
                           1e-4 + 3e-5 * x, -2e-4 + 1e-5 * x, 5e-5 - 4e-5 * x])
            return 1 + 1e-3 + 2e-4 * x, np.zeros(3), sym_to_full(P6[:, None])[:, :, 0]
        return 1.0, np.array([2e-4 + 1e-4 * x, -3e-4 + 4e-5 * x, 1e-4 - 2e-5 * x]), np.zeros((3, 3))

    def box(order, wl, wr):
        return B.slab3(nx, ny, nz, wl, wr, lam=lam, mu=mu, tau=0.55, neumann_order=order)

    probe = Oracle3D(box(1, B.Wall3(B.NEUMANN), B.Wall3(B.NEUMANN)))
    xl, xr = -q_left, nx - 1 + q_right
    if kind == "neumann":
        # sigma = -P at lambda = mu; t* = sigma.n, n = -x at the first wall, +x at the second
        wl = B.Wall3(B.NEUMANN, tuple(fields(xl)[2][:, 0] * probe.s_sigma), q=q_left)
        wr = B.Wall3(B.NEUMANN, tuple(-fields(xr)[2][:, 0] * probe.s_sigma), q=q_right)
    else:
        wl = B.Wall3(B.DIRICHLET, tuple(fields(xl)[1] * probe.s_v), q=q_left)
        wr = B.Wall3(B.DIRICHLET, tuple(fields(xr)[1] * probe.s_v), q=q_right)
    o = Oracle3D(box(1, wl, wr))
    f0 = np.zeros((Q, nz, ny, nx))
    for x in range(nx):
        r, j, P = fields(x)
        f0[:, :, :, x] = equilibrium(np.array([r]), j[:, None], P[:, :, None])[:, 0, None, None]
    o.set_populations(f0)
    o.step(1)
    f1 = o.populations()
    scale = np.abs(f0).max()
    checked = 0
    for i in range(1, Q):
        if C[i, 0] == 0:
            continue
        x = 0 if C[i, 0] < 0 else nx - 1
        r, j, P = fields(x + C[i, 0])                # the virtual site x + c_i
        want = equilibrium(np.array([r]), j[:, None], P[:, :, None])[OPP[i], 0]
        assert np.abs(f1[OPP[i], :, :, x] - want).max() <= 1e-13 * scale, (i, x)
        checked += 1
    assert checked == 10
    if kind == "neumann":
        # rho_bd and the tangential stress at the boundary site (order 0) are not exact
        o0 = Oracle3D(box(0, wl, wr))
        o0.set_populations(f0)
        o0.step(1)
        assert np.abs(o0.populations() - f1).max() > 1e-7 * scale


@pytest.mark.parametrize("q", [0.2, 0.8])
def test_moving_wall_drags_the_material_at_its_velocity(q):
    """A wall crossing the boundary links at q, set moving along y at v_w
    (eq:bbnoncon with j* = rho v_w), launches a shear wave; behind its front
    the material moves with the wall, v = v_w, whatever q (a wrong kappa or
    beta imposes another velocity)."""
    nx, vw = 200, 2e-4
    b = B.slab3(nx, 1, 1, B.Wall3(B.DIRICHLET, (0.0, vw, 0.0), q=q), B.Wall3(B.NEUMANN), lam=0.05, mu=0.05,
                tau=0.55)
    o = Oracle3D(b)
    o.step(int(0.6 * nx * np.sqrt(3)))
    rho, j, P, sig = o.moments()
    v = j[1, 0, 0] / rho[0, 0, 0]
    assert np.mean(v[10:int(0.4 * nx)]) == pytest.approx(vw, rel=0.01)
    assert np.abs(v[int(0.8 * nx):]).max() < 1e-3 * vw


def test_brute_force_loops_on_a_tiny_box():
    """One step of the reference against an explicit per-site loop
    implementation of the same definitions (tests/naive3d.py), on 3 x 4 x 2
    boxes with and without walls, walls at q = 1/2 and elsewhere, rho_bd and
    the tangential stress at the site and extrapolated, and on 1 x 4 x 2
    slabs (both walls on the same sites, no site behind), with random
    populations."""
    rng = np.random.default_rng(8)
    walls2 = (B.Wall3(B.DIRICHLET, (1e-3, 2e-3, -1e-3)), B.Wall3(B.NEUMANN, (2e-4, -1e-4, 3e-4)))
    wallsq = (B.Wall3(B.NEUMANN, (-1e-4, 3e-4, 2e-4), q=0.3), B.Wall3(B.DIRICHLET, (2e-3, -1e-3, 1e-3), q=0.75))
    for nx, walls, order in ((3, None, 0), (3, walls2, 0), (1, walls2, 0), (1, walls2[::-1], 0),
                             (3, wallsq, 0), (3, wallsq, 1), (3, wallsq[::-1], 1), (1, wallsq, 1)):
        b = B.Box3(nx, 4, 2, lam=0.09, mu=0.05, tau=0.6, force=(1e-5, 0.0, -2e-5), x_walls=walls,
                   neumann_order=order)
        o = Oracle3D(b)
        f = o.populations() + rng.normal(size=o.populations().shape) * 1e-3
        o.set_populations(f)
        U0 = rng.normal(size=(3,) + o.shape)
        o.U = U0.copy()
        o.step(1)
        fn, Un = naive_step(b, f, U0, [tuple(int(a) for a in c) for c in C])
        assert np.abs(o.populations() - fn).max() < 1e-14
        assert np.abs(o.U - Un).max() < 1e-14


# ------------------------------------------------ general cut-link geometry --

def _planes_as_links(nx, ny, nz, walls, order, lam=0.09, mu=0.05, tau=0.6):
    """The slab of `walls` (at q_left, q_right) written as a general geometry:
    material columns 1..nx between void columns 0 and nx + 1, periodic in x,
    the links into the void cut at the walls' q with normals -x and +x."""
    NX = nx + 2
    mask = np.zeros((nz, ny, NX), dtype=np.uint8)
    mask[:, :, 1:nx + 1] = 1
    recs = []
    for z in range(nz):
        for y in range(ny):
            for side, x in ((0, 1), (1, nx)):
                for i in range(1, Q):
                    if C[i, 0] == (-1 if side == 0 else 1):
                        recs.append(((z * ny + y) * NX + x, i, walls[side].q, side,
                                     (-1.0 if side == 0 else 1.0, 0.0, 0.0)))
    links = B.link_records3(recs)
    groups = [B.BCGroup3(w.kind, w.value) for w in walls]
    return B.Box3(NX, ny, nz, lam=lam, mu=mu, tau=tau, mask=mask, links=links, groups=groups,
                  neumann_order=order)


@pytest.mark.parametrize("nx,qs,order", [(5, (0.5, 0.5), 0), (5, (0.3, 0.8), 1), (4, (0.9, 0.15), 0),
                                         (1, (0.3, 0.7), 1)])
def test_cut_links_reproduce_the_wall_planes(nx, qs, order):
    """The general geometry (a material mask, per-link q, normal and group)
    reduces to the pinned wall planes: planes written as cut links into void
    columns give the same state (the one-site-wide slab has links with no
    site behind, cut on both sides)."""
    walls = (B.Wall3(B.DIRICHLET, (1e-3, 2e-3, -1e-3), q=qs[0]), B.Wall3(B.NEUMANN, (2e-4, -1e-4, 3e-4), q=qs[1]))
    plane = B.slab3(nx, 4, 3, *walls, lam=0.09, mu=0.05, tau=0.6, neumann_order=order)
    gen = _planes_as_links(nx, 4, 3, walls, order)
    o1, o2 = Oracle3D(plane), Oracle3D(gen)
    rng = np.random.default_rng(11)
    v = 1e-3 * rng.normal(size=(3,) + o1.shape)
    o1.init_fields(vel=v)
    v2 = np.zeros((3,) + o2.shape)
    v2[:, :, :, 1:nx + 1] = v
    o2.init_fields(vel=v2)
    o1.step(9)
    o2.step(9)
    f1, f2 = o1.populations(), o2.populations()[:, :, :, 1:nx + 1]
    assert np.abs(f1 - f2).max() < 1e-14
    assert np.abs(o1.displacement() - o2.displacement()[:, :, :, 1:nx + 1]).max() < 1e-13


@pytest.mark.parametrize("order", [0, 1])
def test_pressurised_cavity_holds_a_hydrostatic_state(order):
    """Patch test of eq:abbnoncon on a curved wall: a spherical cavity under
    pressure p (t* = -p n on every link, each with its own normal) in a
    material under the uniform stress -p I is an exact steady state, at the
    q of every cut link and with the tangential stress at the site or
    extrapolated."""
    p = 2e-4
    b = B.sphere_box3(16, 15, 14, [B.Sphere3(7.3, 6.8, 6.6, 3.7, 0)], [B.BCGroup3(B.NEUMANN, pressure=p)],
                      lam=0.1, mu=0.05, tau=0.6, neumann_order=order)
    assert len(set(np.round(b.links["q"], 6))) > 20
    o = Oracle3D(b)
    sig = np.zeros((6,) + o.shape)
    sig[:3] = -p
    o.init_fields(sigma=sig)
    o.step(6)
    m = o.moments()
    mk = b.mask.astype(bool)
    # rounding leaves ~1e-15; a wrong normal projection errs by the order of p
    assert np.abs(m[3][:, mk] - sig[:, mk]).max() < 1e-13
    assert np.abs(m[1][:, mk]).max() < 1e-13


def test_moving_cavity_carries_a_uniform_translation():
    """Patch test of eq:bbnoncon on a curved wall: a spherical cavity whose
    wall moves with the material's uniform velocity keeps it translating."""
    v0 = np.array([3e-4, -2e-4, 1e-4])
    b = B.sphere_box3(16, 15, 14, [B.Sphere3(7.3, 6.8, 6.6, 3.7, 0)], [B.BCGroup3(B.DIRICHLET, tuple(v0))],
                      lam=0.1, mu=0.05, tau=0.6)
    o = Oracle3D(b)
    o.init_fields(vel=np.broadcast_to(v0[:, None, None, None], (3,) + o.shape))
    o.step(7)
    rho, j, P, sig = o.moments()
    mk = b.mask.astype(bool)
    assert np.abs(j[:, mk] - v0[:, None]).max() < 1e-13
    assert np.abs(sig[:, mk]).max() < 1e-13


@pytest.mark.parametrize("order", [0, 1])
def test_brute_force_loops_with_a_cavity(order):
    """One step of the general geometry against the per-site loop form on a
    6 x 6 x 5 box with a small cavity (links of many q and normals, thin
    links where the cavity is one site across), random populations."""
    b = B.sphere_box3(6, 6, 5, [B.Sphere3(2.6, 2.4, 2.1, 1.3, 0)],
                      [B.BCGroup3(B.NEUMANN, (1e-4, -2e-4, 5e-5), pressure=3e-4)], lam=0.09, mu=0.05, tau=0.6,
                      force=(1e-5, 0.0, -2e-5), neumann_order=order)
    b2 = B.sphere_box3(6, 6, 5, [B.Sphere3(2.6, 2.4, 2.1, 1.3, 0)], [B.BCGroup3(B.DIRICHLET, (1e-3, 2e-3, -1e-3))],
                       lam=0.09, mu=0.05, tau=0.6, neumann_order=order)
    rng = np.random.default_rng(9)
    for box in (b, b2):
        o = Oracle3D(box)
        f = o.populations() + rng.normal(size=o.populations().shape) * 1e-3
        f[:, ~box.mask.astype(bool)] = o.populations()[:, ~box.mask.astype(bool)]
        o.set_populations(f)
        U0 = rng.normal(size=(3,) + o.shape) * box.mask
        o.U = U0.copy()
        o.step(1)
        fn, Un = naive_step(box, f, U0, [tuple(int(a) for a in c) for c in C])
        assert np.abs(o.populations() - fn).max() < 1e-14
        assert np.abs(o.U - Un).max() < 1e-14


def _plane_crack(nx, ny, nz, walls, order, lam=0.09, mu=0.05, tau=0.6):
    """The slab of `walls` (at q_left, q_right) written as a crack of zero
    thickness across a box of nx columns periodic in x, with no void: the
    links between columns nx - 1 and 0 are cut, column 0 seeing the first
    wall (normal -x) and column nx - 1 the second (+x).  With q_left +
    q_right = 1 the two faces are one plane; otherwise each face still sits
    at its own q."""
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    recs = []
    for z in range(nz):
        for y in range(ny):
            for side, x in ((0, 0), (1, nx - 1)):
                for i in range(1, Q):
                    if C[i, 0] == (-1 if side == 0 else 1):
                        recs.append(((z * ny + y) * nx + x, i, walls[side].q, side,
                                     (-1.0 if side == 0 else 1.0, 0.0, 0.0)))
    links = B.link_records3(recs)
    groups = [B.BCGroup3(w.kind, w.value) for w in walls]
    return B.Box3(nx, ny, nz, lam=lam, mu=mu, tau=tau, mask=mask, links=links, groups=groups,
                  neumann_order=order)


@pytest.mark.parametrize("nx,qs,order", [(5, (0.5, 0.5), 0), (6, (0.3, 0.7), 1), (4, (0.9, 0.15), 0)])
def test_plane_crack_reproduces_the_wall_planes(nx, qs, order):
    """Cut links between two material sites (a crack, both faces listed)
    reduce to the pinned wall planes: a crack across a box periodic in x,
    without any void, gives the state of the slab with the two walls."""
    walls = (B.Wall3(B.NEUMANN, (-1e-4, 3e-4, 0.0), q=qs[0]), B.Wall3(B.DIRICHLET, (1e-3, 2e-3, -1e-3), q=qs[1]))
    plane = B.slab3(nx, 4, 3, *walls, lam=0.09, mu=0.05, tau=0.6, neumann_order=order)
    crack = _plane_crack(nx, 4, 3, walls, order)
    o1, o2 = Oracle3D(plane), Oracle3D(crack)
    rng = np.random.default_rng(12)
    v = 1e-3 * rng.normal(size=(3,) + o1.shape)
    o1.init_fields(vel=v)
    o2.init_fields(vel=v)
    o1.step(9)
    o2.step(9)
    assert np.abs(o1.populations() - o2.populations()).max() < 1e-14
    assert np.abs(o1.displacement() - o2.displacement()).max() < 1e-13


def _penny(order, groups, lam=0.1):
    return B.sphere_box3(14, 13, 10, [], groups, lam=lam, mu=0.05, tau=0.6, neumann_order=order,
                         cracks=[B.PennyCrack3(6.6, 6.2, 4.3, 4.1, 0, 1)])


@pytest.mark.parametrize("order", [0, 1])
def test_penny_crack_leaves_an_in_plane_stress_alone(order):
    """Patch test of eq:abbnoncon at a crack: traction-free faces normal to z
    carry no load under a uniform stress in the crack's plane (sigma_xx,
    sigma_yy, sigma_xy), which is therefore an exact steady state; a
    crack that transmitted normal or shear stress, or a wrong q, would
    disturb it by the order of the stress."""
    b = _penny(order, [B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN)])
    assert len(b.links) > 100 and b.n_material == b.n_sites
    o = Oracle3D(b)
    sig = np.zeros((6,) + o.shape)
    sig[0], sig[1], sig[3] = 3e-4, -1e-4, 2e-4
    o.init_fields(sigma=sig)
    o.step(8)
    m = o.moments()
    assert np.abs(m[3] - sig).max() < 1e-13
    assert np.abs(m[1]).max() < 1e-13


def test_penny_crack_opens_under_normal_tension():
    """The same crack under a normal tension sigma_zz (traction-free faces):
    the faces move apart (the material below moves down, above moves up),
    unlike the uncracked box, which stays at rest."""
    b = _penny(0, [B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN)])
    o = Oracle3D(b)
    sig = np.zeros((6,) + o.shape)
    sig[2] = 2e-4
    o.init_fields(sigma=sig)
    o.step(12)
    u = o.displacement()
    uz_below, uz_above = u[2, 4, 6, 6], u[2, 5, 6, 6]            # either side of the crack's centre
    assert uz_below < -1e-6 and uz_above > 1e-6
    ref = Oracle3D(B.periodic_box3(14, 13, 10, lam=0.1, mu=0.05, tau=0.6))
    ref.init_fields(sigma=sig)
    ref.step(12)
    assert np.abs(ref.displacement()).max() < 1e-15


@pytest.mark.parametrize("order", [0, 1])
def test_brute_force_loops_with_a_crack(order):
    """One step with a penny crack (both faces, with pressure and shear
    traction, and a moving face) against the per-site loop form."""
    b = B.sphere_box3(7, 7, 5, [], [B.BCGroup3(B.NEUMANN, (1e-4, -2e-4, 5e-5), pressure=3e-4),
                                  B.BCGroup3(B.DIRICHLET, (1e-3, 2e-3, -1e-3))],
                      lam=0.09, mu=0.05, tau=0.6, force=(1e-5, 0.0, -2e-5), neumann_order=order,
                      cracks=[B.PennyCrack3(3.1, 2.9, 2.35, 1.8, 0, 1)])
    assert len(b.links) > 10
    rng = np.random.default_rng(10)
    o = Oracle3D(b)
    f = o.populations() + rng.normal(size=o.populations().shape) * 1e-3
    o.set_populations(f)
    U0 = rng.normal(size=(3,) + o.shape)
    o.U = U0.copy()
    o.step(1)
    fn, Un = naive_step(b, f, U0, [tuple(int(a) for a in c) for c in C])
    assert np.abs(o.populations() - fn).max() < 1e-14
    assert np.abs(o.U - Un).max() < 1e-14


def test_one_sided_crack_is_refused():
    b = _penny(0, [B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN)])
    lower = b.links[b.links["group"] == 0]
    b.links = lower                                  # the upper face missing
    with pytest.raises(ValueError):
        Oracle3D(b)


FACES = [(-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, -1.0), (0.0, 0.0, 1.0)]


def _block(groups, order, lam=0.065):
    """A 5 x 4 x 4 block in an 8 x 7 x 7 periodic box, one group per face."""
    return B.block_box3(8, 7, 7, (1, 2, 1), (5, 5, 4), list(range(6)), groups, lam=lam, mu=0.05, tau=0.6,
                        neumann_order=order)


@pytest.mark.parametrize("order", [0, 1])
def test_block_holds_a_uniform_stress(order):
    """Patch test of the rules on a block's faces, edges included: every face
    loaded by the traction sigma.n of one uniform stress sigma (all six
    components non-zero) keeps that stress exactly.  At the edges the links
    carry two faces' groups and normals; a wrong combination of the two
    tractions (their shear, or the edge's own component) disturbs it by the
    order of sigma."""
    sig3 = np.array([[3e-4, 1e-4, -2e-4], [1e-4, -1e-4, 1.5e-4], [-2e-4, 1.5e-4, 2e-4]])
    groups = [B.BCGroup3(B.NEUMANN, tuple(sig3 @ np.array(n))) for n in FACES]
    b = _block(groups, order)
    assert (b.links["group2"] >= 0).sum() > 20
    o = Oracle3D(b)
    sig = np.zeros((6,) + o.shape)
    for k, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        sig[k] = sig3[i, j]
    # a uniform density change too: the (lambda - mu) drho terms of the rules
    o.init_fields(rho=np.full(o.shape, 1.0 + 3e-4), sigma=sig)
    o.step(8)
    m = o.moments()
    mk = b.mask.astype(bool)
    assert np.abs(m[3][:, mk] - sig[:, mk]).max() < 1e-13
    assert np.abs(m[1][:, mk]).max() < 1e-13


def test_block_with_a_moving_face_translates():
    """A block moving at v0 with one Dirichlet face (wall velocity v0) and
    five traction-free faces keeps its uniform translation: at the edges of
    the moving face the Dirichlet face wins."""
    v0 = np.array([2e-4, -1e-4, 3e-4])
    groups = [B.BCGroup3(B.DIRICHLET, tuple(v0))] + [B.BCGroup3(B.NEUMANN)] * 5
    b = _block(groups, 0)
    o = Oracle3D(b)
    o.init_fields(vel=np.broadcast_to(v0[:, None, None, None], (3,) + o.shape))
    o.step(7)
    rho, j, P, sg = o.moments()
    mk = b.mask.astype(bool)
    assert np.abs(j[:, mk] - v0[:, None]).max() < 1e-13
    assert np.abs(sg[:, mk]).max() < 1e-13


@pytest.mark.parametrize("order", [0, 1])
def test_brute_force_loops_with_a_block(order):
    """One step of a block with faces of both kinds, loaded and moving (edges
    of two Neumann faces, of two Dirichlet faces and of one of each) against
    the per-site loop form."""
    groups = [B.BCGroup3(B.NEUMANN, (1e-4, -2e-4, 5e-5), pressure=3e-4), B.BCGroup3(B.DIRICHLET, (1e-3, 0.0, -1e-3)),
              B.BCGroup3(B.NEUMANN, (0.0, 2e-4, 1e-4)), B.BCGroup3(B.DIRICHLET, (-1e-3, 2e-3, 0.0)),
              B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN, (3e-4, 0.0, 0.0), pressure=-1e-4)]
    b = B.block_box3(6, 6, 6, (1, 1, 1), (4, 3, 4), list(range(6)), groups, lam=0.09, mu=0.05, tau=0.6,
                     force=(1e-5, 0.0, -2e-5), neumann_order=order)
    rng = np.random.default_rng(13)
    o = Oracle3D(b)
    f = o.populations() + rng.normal(size=o.populations().shape) * 1e-3
    f[:, ~b.mask.astype(bool)] = o.populations()[:, ~b.mask.astype(bool)]
    o.set_populations(f)
    U0 = rng.normal(size=(3,) + o.shape) * b.mask
    o.U = U0.copy()
    o.step(1)
    fn, Un = naive_step(b, f, U0, [tuple(int(a) for a in c) for c in C])
    assert np.abs(o.populations() - fn).max() < 1e-14
    assert np.abs(o.U - Un).max() < 1e-14


def _ramped(make, T_steps, step):
    """Oracle on make(profile kwargs), populations at a random state, its
    step counter at `step`: one step."""
    rng = np.random.default_rng(17)
    b = make()
    o = Oracle3D(b)
    f = o.populations() + rng.normal(size=o.populations().shape) * 1e-3
    if b.mask is not None:
        f[:, ~b.mask.astype(bool)] = o.populations()[:, ~b.mask.astype(bool)]
    o.set_populations(f)
    o.n = step
    o.step(1)
    return o.populations()


@pytest.mark.parametrize("geometry", ["walls", "links"])
def test_ramped_values_take_the_time_of_the_step(geometry):
    """A RAMP profile scales a wall's or group's value by min(t_n / T, 1), t_n
    the time of the post-collision state the rule reads: from the same state,
    one step at n = 0 equals the step with the value zero, at n = 3 of a
    10-step ramp the step with 0.3 of the value, and past the ramp the STEP
    profile's step."""
    dt = np.sqrt(1.0 / (3 * 0.05))
    T = 10 * dt
    vd, vn = (1e-3, -2e-3, 5e-4), (2e-4, 1e-4, -3e-4)

    def make(scale=1.0, ramp=True):
        kw = dict(profile=B.RAMP, ramp_time=T) if ramp else {}
        if geometry == "walls":
            return B.slab3(5, 4, 3, B.Wall3(B.DIRICHLET, tuple(scale * v for v in vd), q=0.3, **kw),
                           B.Wall3(B.NEUMANN, tuple(scale * v for v in vn), q=0.8, **kw), lam=0.09, mu=0.05,
                           tau=0.6, neumann_order=1)
        groups = [B.BCGroup3(B.NEUMANN, tuple(scale * v for v in vn), scale * 2e-4, **kw),
                  B.BCGroup3(B.DIRICHLET, tuple(scale * v for v in vd), **kw)]
        return B.sphere_box3(8, 7, 7, [B.Sphere3(3.4, 3.2, 3.1, 1.7, 0)], groups, lam=0.09, mu=0.05, tau=0.6,
                             neumann_order=1, cracks=[])

    ref0 = _ramped(lambda: make(0.0, False), 10, 0)
    assert np.abs(_ramped(make, 10, 0) - ref0).max() == 0.0
    assert np.abs(_ramped(make, 10, 3) - _ramped(lambda: make(0.3, False), 10, 3)).max() < 1e-17
    assert np.abs(_ramped(make, 10, 14) - _ramped(lambda: make(1.0, False), 10, 14)).max() == 0.0
    assert np.abs(_ramped(make, 10, 3) - ref0).max() > 1e-6


@pytest.mark.parametrize("order", [0, 1])
def test_brute_force_loops_with_ramped_groups(order):
    """One step at step index 4 of ramped walls and groups against the
    per-site loop form (which applies the profile itself)."""
    dt = np.sqrt(1.0 / (3 * 0.05))
    rng = np.random.default_rng(19)
    boxes = [B.slab3(4, 4, 3, B.Wall3(B.DIRICHLET, (1e-3, 2e-3, -1e-3), q=0.3, profile=B.RAMP, ramp_time=9 * dt),
                     B.Wall3(B.NEUMANN, (2e-4, -1e-4, 3e-4), q=0.7, profile=B.RAMP, ramp_time=6 * dt),
                     lam=0.09, mu=0.05, tau=0.6, neumann_order=order),
             B.sphere_box3(6, 6, 5, [B.Sphere3(2.6, 2.4, 2.1, 1.3, 0)],
                           [B.BCGroup3(B.NEUMANN, (1e-4, -2e-4, 5e-5), 3e-4, profile=B.RAMP, ramp_time=7 * dt)],
                           lam=0.09, mu=0.05, tau=0.6, neumann_order=order)]
    for box in boxes:
        o = Oracle3D(box)
        f = o.populations() + rng.normal(size=o.populations().shape) * 1e-3
        if box.mask is not None:
            f[:, ~box.mask.astype(bool)] = o.populations()[:, ~box.mask.astype(bool)]
        o.set_populations(f)
        U0 = rng.normal(size=(3,) + o.shape) * (1 if box.mask is None else box.mask)
        o.U = U0.copy()
        o.n = 4
        o.step(1)
        fn, Un = naive_step(box, f, U0, [tuple(int(a) for a in c) for c in C], step=4)
        assert np.abs(o.populations() - fn).max() < 1e-14
        assert np.abs(o.U - Un).max() < 1e-14


def test_inconsistent_cut_links_are_refused():
    b = B.sphere_box3(10, 9, 8, [B.Sphere3(4.4, 4.2, 3.9, 2.2, 0)], [B.BCGroup3(B.NEUMANN)])
    for bad in ("missing", "material_far_end", "q"):
        links = b.links.copy()
        if bad == "missing":
            links = links[1:]
        elif bad == "material_far_end":
            links["dir"][0] = B.C3.tolist().index([-c for c in B.C3[links["dir"][0]].tolist()])
        else:
            links["q"][0] = 1.5
        with pytest.raises(ValueError):
            Oracle3D(B.Box3(b.nx, b.ny, b.nz, lam=b.lam, mu=b.mu, tau=b.tau, mask=b.mask, links=links,
                            groups=b.groups))
