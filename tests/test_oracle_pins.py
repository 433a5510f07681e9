"""Pins of the CPU reference against what the paper and the mathematics fix.

Each test names the property and the passage it comes from.  None of them
re-types the reference's formulas: they check moment identities, exact
invariants, closed-form wave speeds, exact uniform solutions, symmetry, a
second formulation of the step in moment space, and numbers the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import Oracle, equilibrium
from slbm_workloads import geometry as G
from slbm_workloads import configs
import closed_forms as CF
from naive_moment_lbm import NaiveLBM

HERE = os.path.dirname(os.path.abspath(__file__))
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def moments_of(f):
    """rho, j, P of populations f[9, ...] (eq:moments without the S/2 part)."""
    rho = f.sum(0)
    jx = np.tensordot(CX, f, 1)
    jy = np.tensordot(CY, f, 1)
    pxx = np.tensordot(CX * CX, f, 1)
    pyy = np.tensordot(CY * CY, f, 1)
    pxy = np.tensordot(CX * CY, f, 1)
    return rho, jx, jy, pxx, pyy, pxy


# ------------------------------------------------------------- eq:fieq --

def test_equilibrium_has_the_prescribed_moments():
    """eq:fieq is built so that its moments are rho, j and P (section 3)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        j = 0.05 * rng.standard_normal(2)
        P = 0.05 * rng.standard_normal(3)
        f = equilibrium(rho, j, P)
        r, jx, jy, pxx, pyy, pxy = moments_of(f[:, None])
        np.testing.assert_allclose([r[0], jx[0], jy[0], pxx[0], pyy[0], pxy[0]],
                                   [rho, j[0], j[1], P[0], P[1], P[2]], atol=1e-15, rtol=1e-14)


def test_rest_equilibrium_is_the_unstressed_state():
    """At rest (rho = 1, j = 0, no stress) the Poisson stress is zero
    (eq:poissonstress), so f_eq = w_i (2 - 3|c_i|^2/2)."""
    f = equilibrium(1.0, np.zeros(2), np.zeros(3))
    expect = [8 / 9] + [1 / 18] * 4 + [-1 / 36] * 4
    np.testing.assert_allclose(f, expect, rtol=0, atol=1e-16)


# ------------------------------------------------------------- eq:coll --

def test_collision_conserves_rho_and_P_and_adds_S_to_momentum():
    """With eq:moments, BGK with the forcing of eq:coll leaves rho and P
    unchanged and raises sum f c by exactly S.  On a 1x1 periodic lattice the
    streaming maps every population onto itself and grad rho = 0, so S = F."""
    F = (2e-4, -3e-4)
    p = G.periodic_box(1, 1, lam=0.07, mu=0.05, tau=0.55, force=F)
    o = Oracle(p)
    rng = np.random.default_rng(2)
    f0 = equilibrium(1.0, np.zeros(2), np.zeros(3)) + 1e-3 * rng.standard_normal(9)
    o.set_populations(f0.reshape(9, 1, 1))
    o.step(1)
    f1 = o.populations()[:, 0, 0]
    m0 = moments_of(f0[:, None])
    m1 = moments_of(f1[:, None])
    S = np.array(F) / (3 * 0.05)
    assert abs(m1[0][0] - m0[0][0]) < 1e-15
    np.testing.assert_allclose([m1[3][0], m1[4][0], m1[5][0]], [m0[3][0], m0[4][0], m0[5][0]], atol=1e-15)
    np.testing.assert_allclose([m1[1][0] - m0[1][0], m1[2][0] - m0[2][0]], S, rtol=1e-12, atol=1e-17)


# ------------------------------------------------------ invariants --

def test_periodic_mass_conservation():
    """Streaming and collision conserve sum rho exactly in a periodic box
    (eq:coll, eq:stream), for any lambda/mu."""
    p = G.periodic_box(24, 20, lam=0.08, mu=0.05, tau=0.6)
    o = Oracle(p, extended=True)
    rng = np.random.default_rng(3)
    o.init_fields(rho=1 + 1e-3 * rng.standard_normal((20, 24)),
                  vel=1e-3 * rng.standard_normal((2, 20, 24)))
    m0 = o.moments()[0].sum()
    o.step(50)
    assert abs(o.moments()[0].sum() - m0) < 1e-12 * m0


def test_periodic_momentum_conservation_when_lambda_equals_mu():
    """With lambda = mu the source term is F alone (eq:sourceterm), so in a
    periodic box sum j changes by exactly N F per step."""
    for F in [(0.0, 0.0), (3e-6, -2e-6)]:
        p = G.periodic_box(16, 12, lam=0.05, mu=0.05, tau=0.55, force=F)
        o = Oracle(p, extended=True)
        rng = np.random.default_rng(4)
        o.init_fields(vel=1e-3 * rng.standard_normal((2, 12, 16)),
                      sigma=1e-4 * rng.standard_normal((3, 12, 16)))
        j0 = o.moments()[1].sum(axis=(1, 2))
        o.step(40)
        j1 = o.moments()[1].sum(axis=(1, 2))
        # user units: j changes by F * dt per step and site
        dt = math.sqrt(1.0 / (3 * 0.05))
        np.testing.assert_allclose(j1 - j0, 16 * 12 * 40 * dt * np.array(F), atol=1e-13)


# ---------------------------------------------- closed-form wave speeds --

def _phase_speed(lam, mu, tau, pol):
    """Phase speed of a plane wave k = 2 pi/64 along x in a periodic box,
    from the zero crossings of the velocity amplitude (in cells per step)."""
    n = 64
    p = G.periodic_box(n, 1, lam=lam, mu=mu, tau=tau)
    o = Oracle(p)
    x = np.arange(n)
    v = np.zeros((2, 1, n))
    v[pol, 0] = 1e-4 * np.sin(2 * np.pi * x / n)
    o.init_fields(vel=v)
    s = np.sin(2 * np.pi * x / n)
    amp = []
    for _ in range(1400):
        o.step(1)
        amp.append(np.dot(o.moments()[1][pol, 0], s))
    amp = np.array(amp)
    t = np.arange(1, len(amp) + 1)
    z = [t[i] - amp[i] / (amp[i + 1] - amp[i]) for i in range(len(amp) - 1) if amp[i] * amp[i + 1] < 0]
    half = np.diff(z)[2:].mean()          # skip the first crossings (start-up)
    omega = np.pi / half
    return omega / (2 * np.pi / n)


@pytest.mark.parametrize("lam_over_mu,tau", [(1.0, 0.55), (0.769, 0.55), (2.0, 0.6)])
def test_plane_wave_speeds_match_the_lame_navier_equation(lam_over_mu, tau):
    """Lame-Navier (eq:navier): c_s^2 = mu/rho, c_d^2 = (lambda + 2 mu)/rho.
    In lattice units mu = 1/3 (c_s^2 = 1/3, section 5.1)."""
    mu_L, lam_L = 1 / 3, lam_over_mu / 3
    cs, cd = CF.wave_speeds(lam_L, mu_L)
    c_p = _phase_speed(lam_over_mu * 0.05, 0.05, tau, pol=0)
    c_s = _phase_speed(lam_over_mu * 0.05, 0.05, tau, pol=1)
    assert abs(c_p / cd - 1) < 1e-3, (c_p, cd)
    assert abs(c_s / cs - 1) < 1e-3, (c_s, cs)


# ------------------------------------------------- exact uniform states --

def _patch_plate(neumann_order, with_dirichlet):
    """A plate with straight edges and an off-centre circular hole: every
    kind of link (q = 1/2, q in (0,1), corners, diagonals)."""
    n = 30
    walls = G.edge_walls(n, n, left=0, right=1, bottom=2, top=3)
    walls.append(G.Circle(13.3, 15.8, 5.7, 4))
    groups = [G.BCGroup(G.NEUMANN)] * 5
    p = G.build_plate(n, n, lam=0.08, mu=0.05, tau=0.55, walls=walls, groups=groups,
                      neumann_order=neumann_order)
    return p


@pytest.mark.parametrize("neumann_order", [1, 0])
@pytest.mark.parametrize("with_dirichlet", [False, True])
def test_uniform_state_with_consistent_boundary_data_is_exact(neumann_order, with_dirichlet):
    """A uniform state (rho0, j0, sigma0) solves the moment chain exactly.
    With j* = j0 on Dirichlet links and t* = sigma0 n on Neumann links, the
    bounce-back rules reproduce it for every wall fraction q (the Bouzidi-type
    terms cancel because l - 2s and 2l enter as (l-2s)/(l+2s) - 2l/(l+2s) = -1),
    and the displacement grows as t * j0/rho0.  Exact up to rounding."""
    p = _patch_plate(neumann_order, with_dirichlet)
    rho0, v0 = 1.0 + 2e-3, np.array([3e-4, -2e-4])
    sig0 = np.array([[4e-5, -1.5e-5], [-1.5e-5, 2.5e-5]])
    L = p.links.copy()
    groups = []
    rng = np.random.default_rng(5)
    for i in range(len(L)):
        # a random mix of Dirichlet and Neumann links, each with its own data
        dirichlet = with_dirichlet and rng.uniform() < 0.5
        if dirichlet:
            groups.append(G.BCGroup(G.DIRICHLET, tuple(v0)))
        else:
            groups.append(G.BCGroup(G.NEUMANN, tuple(sig0 @ L["normal"][i])))
        L["group"][i] = len(groups) - 1
        if L["group2"][i] >= 0:
            groups.append(G.BCGroup(G.NEUMANN, tuple(sig0 @ L["normal2"][i])))
            L["group2"][i] = len(groups) - 1
    p.links, p.groups = L, groups
    o = Oracle(p, extended=True)
    m = p.mask
    o.init_fields(rho=np.where(m, rho0, 1.0), vel=v0[:, None, None] * m,
                  sigma=np.array([sig0[0, 0], sig0[1, 1], sig0[0, 1]])[:, None, None] * m)
    f0 = o.populations()
    o.step(25)
    f1 = o.populations()
    assert np.abs(f1 - f0).max() < 1e-15
    u = o.displacement()
    dt = math.sqrt(1 / (3 * 0.05))
    np.testing.assert_allclose(u[:, m.astype(bool)], (25 * v0 * dt)[:, None] * np.ones((2, int(m.sum()))),
                               rtol=1e-12)


# --------------------------------------------------------- symmetry --

def _loaded_plate(order):
    n = 36
    groups = [G.BCGroup(G.DIRICHLET, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (1e-3 * 0.05, 0.0)),
              G.BCGroup(G.NEUMANN, (0.0, 0.0))]
    walls = G.edge_walls(n, n, left=0, right=1, bottom=2, top=2)
    walls.append(G.Circle(20.2, (n - 1) / 2, 6.3, 2))
    return G.build_plate(n, n, lam=0.04, mu=0.05, tau=0.55, walls=walls, groups=groups,
                         neumann_order=order)


@pytest.mark.parametrize("order", [1, 0])
def test_mirror_symmetry(order):
    """The step commutes with reflection about the mid-line: a problem
    symmetric about y = (ny-1)/2 keeps u_x even and u_y odd."""
    p = _loaded_plate(order)
    o = Oracle(p)
    o.step(120)
    u = o.displacement()
    scale = np.abs(u).max()
    assert scale > 1e-4
    np.testing.assert_allclose(u[0], u[0, ::-1], atol=1e-11 * scale)
    np.testing.assert_allclose(u[1], -u[1, ::-1], atol=1e-11 * scale)


def test_rotation_equivariance():
    """Rotating the problem by 90 degrees rotates the solution."""
    p = _loaded_plate(1)
    walls = G.edge_walls(p.nx, p.ny, left=0, right=1, bottom=2, top=2)
    walls.append(G.Circle(20.2, 13.1, 6.3, 2))    # break the mirror symmetry
    p = G.build_plate(p.nx, p.ny, lam=0.04, mu=0.05, tau=0.55, walls=walls, groups=p.groups)
    q = G.rotate90(p)
    a, b = Oracle(p), Oracle(q)
    a.step(80)
    b.step(80)
    ua, ub = a.displacement(), b.displacement()
    # rotated field: ub[:, x, ny-1-y] = R ua[:, y, x], R (ux, uy) = (-uy, ux)
    yy, xx = np.mgrid[0:p.ny, 0:p.nx]
    rot = np.empty_like(ub)
    rot[0][xx, p.ny - 1 - yy] = -ua[1]
    rot[1][xx, p.ny - 1 - yy] = ua[0]
    scale = np.abs(ua).max()
    np.testing.assert_allclose(ub, rot, atol=1e-11 * scale)


# ------------------------------------------- second formulation, tiny --

def _tiny_plate(seed):
    rng = np.random.default_rng(seed)
    n = 9
    groups = []
    for _ in range(6):
        if rng.uniform() < 0.4:
            groups.append(G.BCGroup(G.DIRICHLET, tuple(1e-3 * rng.standard_normal(2)),
                                    int(rng.integers(0, 2)), float(rng.uniform(3, 20))))
        else:
            groups.append(G.BCGroup(G.NEUMANN, tuple(1e-4 * rng.standard_normal(2)),
                                    int(rng.integers(0, 2)), float(rng.uniform(3, 20))))
    walls = G.edge_walls(n, n, left=0, right=1, bottom=2, top=3)
    walls.append(G.Circle(rng.uniform(3.5, 5.5), rng.uniform(3.5, 5.5), rng.uniform(1.2, 2.2), 4))
    walls.append(G.HLine(7.5, 5, x_lo=-0.5, x_hi=float(rng.integers(2, 5)) - 0.5))
    return G.build_plate(n, n, lam=rng.uniform(0.5, 2.0) * 0.05, mu=0.05, rho=rng.uniform(0.8, 1.5),
                         tau=0.6, walls=walls, groups=groups, force=tuple(1e-5 * rng.standard_normal(2)),
                         neumann_order=int(seed % 2))


@pytest.mark.parametrize("seed", range(6))
def test_reference_agrees_with_moment_space_formulation(seed):
    """The population-space reference and an independent moment-space,
    dict-of-sites formulation of the same step agree on tiny random plates
    (curved and straight walls, a crack slit, corners, both rule kinds, step
    and ramp profiles, body force) to rounding."""
    p = _tiny_plate(seed)
    o = Oracle(p)
    nv = NaiveLBM(p)
    rng = np.random.default_rng(100 + seed)
    f0 = o.populations() + 1e-3 * rng.standard_normal((9, p.ny, p.nx)) * p.mask
    o.set_populations(f0)
    nv.set_f(f0)
    for _ in range(12):
        o.step(1)
        nv.step()
    np.testing.assert_allclose(o.populations(), nv.get_f(), atol=2e-14)


# ------------------------------------------------- 1-D step traction --

OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


@pytest.mark.parametrize("kind", ["neumann", "dirichlet"])
@pytest.mark.parametrize("q_bottom,q_top", [(0.5, 0.5), (0.3, 0.8), (0.9, 0.15)])
def test_boundary_rules_are_exact_for_linear_fields(kind, q_bottom, q_top):
    """Section 4.2: the interpolated rules are built so that, for an
    equilibrium field varying linearly across the wall, the population a cut
    link returns equals the one the lattice would have streamed in from the
    virtual site x + c_k had the field continued -- for every q.  For the
    Neumann rule (j = 0) this needs the linear extrapolation of rho_bd and
    sigma_tt along the link (neumann_order 1); for the Dirichlet rule, a
    linear velocity field with the wall velocity at the wall point.  Walls are
    horizontal lines at y = -q_bottom and y = ny - 1 + q_top."""
    nx, ny = 6, 5
    lam = mu = 0.05
    if kind == "neumann":
        def fields(y):      # lattice units: rho, j, P (xx, yy, xy)
            return 1 + 1e-3 + 2e-4 * y, (0.0, 0.0), (3e-4 - 1e-4 * y, 2e-4 + 5e-5 * y, 1e-4 + 3e-5 * y)
        g_bot = G.BCGroup(G.NEUMANN, (0.0, 0.0))
        g_top = G.BCGroup(G.NEUMANN, (0.0, 0.0))
    else:
        def fields(y):
            return 1.0, (2e-4 + 1e-4 * y, -3e-4 + 4e-5 * y), (0.0, 0.0, 0.0)
        g_bot = G.BCGroup(G.DIRICHLET, (0.0, 0.0))
        g_top = G.BCGroup(G.DIRICHLET, (0.0, 0.0))
    walls = [G.HLine(-q_bottom, 0), G.HLine(ny - 1 + q_top, 1)]
    plate0 = G.build_plate(nx, ny, lam=lam, mu=mu, tau=0.55, walls=walls, groups=[g_bot, g_top],
                           periodic_x=True, neumann_order=1)
    par = Oracle(plate0).lattice_params()
    # boundary data of the linear field at the wall points, in user units
    yb, yt = -q_bottom, ny - 1 + q_top
    if kind == "neumann":
        # sigma = -P at lambda = mu; t = sigma.n with n = (0, -1) below, (0, 1) above
        _, _, Pb = fields(yb)
        _, _, Pt = fields(yt)
        g_bot.value = (Pb[2] * par["s_sigma"], Pb[1] * par["s_sigma"])
        g_top.value = (-Pt[2] * par["s_sigma"], -Pt[1] * par["s_sigma"])
    else:
        g_bot.value = tuple(v * par["s_v"] for v in fields(yb)[1])
        g_top.value = tuple(v * par["s_v"] for v in fields(yt)[1])
    plate = G.build_plate(nx, ny, lam=lam, mu=mu, tau=0.55, walls=walls, groups=[g_bot, g_top],
                          periodic_x=True, neumann_order=1)
    assert sorted(set(plate.links["q"].round(12))) == sorted({round(q_bottom, 12), round(q_top, 12)})
    o = Oracle(plate)
    f0 = np.zeros((9, ny, nx))
    for y in range(ny):
        r, j, P = fields(y)
        f0[:, y, :] = equilibrium(r, j, P)[:, None]
    o.set_populations(f0)
    o.step(1)
    f1 = o.populations()
    scale = np.abs(f0).max()
    checked = 0
    for L in plate.links:
        x, y = int(L["site"]) % nx, int(L["site"]) // nx
        k = int(L["dir"])
        r, j, P = fields(y + CY[k])                 # the virtual site x + c_k
        want = equilibrium(r, j, P)[OPP[k]]
        assert abs(f1[OPP[k], y, x] - want) <= 1e-13 * scale, (x, y, k)
        checked += 1
    assert checked == 2 * 3 * nx
    if kind == "neumann":
        # the boundary-site values of rho_bd and sigma_tt (order 0) are not exact
        plate.neumann_order = 0
        o0 = Oracle(plate)
        o0.set_populations(f0)
        o0.step(1)
        d = np.abs(o0.populations() - f1).max()
        assert d > 1e-7 * scale


def test_step_traction_launches_the_dilatational_wave():
    """A strip pulled at one end by a step traction sigma0 carries a
    dilatational wave with particle velocity sigma0/(rho c_d) behind the
    front, moving at c_d; at a clamped end the stress doubles."""
    nx, ny = 200, 2
    mu, lam, load = 0.05, 0.05, 1e-4 * 0.05
    groups = [G.BCGroup(G.DIRICHLET, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (load, 0.0))]
    p = G.build_plate(nx, ny, lam=lam, mu=mu, tau=0.55,
                      walls=G.edge_walls(nx, ny, left=0, right=1), groups=groups, periodic_y=True)
    o = Oracle(p)
    cd = math.sqrt((lam + 2 * mu) / 1.0)        # user units (dx = 1)
    dt = math.sqrt(1.0 / (3 * mu))
    steps = 100                                  # c_d = 1 cell per step for lambda = mu
    o.step(steps)
    rho, j, P, s = o.moments()
    front = nx - 1 - steps * cd * dt
    behind = slice(int(front) + 15, nx - 15)
    v = j[0, 0, behind]
    # the pulled end moves outward: v = +sigma0/(rho c_d) behind a tensile
    # wave travelling toward -x ...
    np.testing.assert_allclose(v, load / cd, rtol=2e-2)
    np.testing.assert_allclose(s[0, 0, behind], load, rtol=2e-2)
    ahead = slice(0, int(front) - 15)
    assert np.abs(j[0, 0, ahead]).max() < 1e-3 * load / cd
    # ... and after reflection at the clamped end the stress there doubles
    o.step(220)
    rho, j, P, s = o.moments()
    np.testing.assert_allclose(s[0, 0, 5:40], 2 * load, rtol=3e-2)


# ------------------------------------------------ unit mapping (paper) --

def test_time_step_matches_the_paper():
    """(1/sqrt 3) dx/dt = c_s with dx = 0.0125 l gives dt = 7.217e-3 l/c_s
    (section 5.1), and the speed ratios give the printed Poisson ratios."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))
    p = configs.paper_hole_plate(3.0)
    o = Oracle(p)
    dt = o.lattice_params()["dt_user"]
    l = p.nx * 1.0          # dx = 1 cell = 0.0125 l
    cs = math.sqrt(p.mu / p.rho)
    assert abs(dt * cs / l - g["hole_plate_dt_over_l_per_cs"]["value"]) < 5e-7
    assert abs(CF.nu_from_speed_ratio(g["poisson_solid"]["cd2_over_cs2"]) - g["poisson_solid"]["nu"]) < 1e-12
    assert abs(CF.nu_from_speed_ratio(g["non_poisson_solid"]["cd2_over_cs2"]) - g["non_poisson_solid"]["nu"]) < 1e-12
    assert abs(CF.nu_from_speed_ratio(1 / g["crack_solid"]["cs2_over_cd2"]) - g["crack_solid"]["nu"]) < 1e-4


def test_rayleigh_root_closed_form():
    """The Rayleigh equation the paper solves for the surface-wave speed has
    the classical root c_R = 0.9194 c_s at nu = 1/4."""
    cs, cd = CF.wave_speeds(1.0, 1.0)
    assert abs(CF.rayleigh_speed(cs, cd) / cs - 0.91940) < 1e-5


def test_domain_of_dependence_is_two_columns_per_step():
    """A step reads neighbours one site away (the pull) and the density of
    the pulled state one site further (the source term's gradient), so after
    k steps a site depends only on sites within 2k columns.  A 256-wide plate
    pulled on its right edge and a 64-wide plate with the same edges then
    agree exactly in their right-most 64 - 2k - 2 columns, and sites farther
    than 2k columns from the pulled edge are exactly as in the same plate
    without the load (at rest up to the rounding of the unshifted rest
    populations, which both share)."""
    n, k, w = 256, 10, 64
    full = configs.square_clamped_pulled(n, steps=k)
    crop = G.build_plate(w, n, lam=full.lam, mu=full.mu, tau=full.tau,
                         walls=G.edge_walls(w, n, left=0, right=1, bottom=2, top=2), groups=full.groups,
                         neumann_order=full.neumann_order, name="crop")
    a, b = Oracle(full), Oracle(crop)
    a.step(k)
    b.step(k)
    ua, ub = a.displacement(), b.displacement()
    m = w - 2 * k - 2
    assert np.abs(ub[:, :, w - m:]).max() > 0
    assert np.array_equal(ua[:, :, n - m:], ub[:, :, w - m:])
    rest = G.build_plate(n, n, lam=full.lam, mu=full.mu, tau=full.tau,
                         walls=G.edge_walls(n, n, left=0, right=1, bottom=2, top=2),
                         groups=[full.groups[0], G.BCGroup(G.NEUMANN, (0.0, 0.0)), full.groups[2]],
                         neumann_order=full.neumann_order, name="rest")
    r = Oracle(rest)
    r.step(k)
    u0 = r.displacement()
    far = n - 2 * k - 1
    assert np.array_equal(ua[:, :, :far], u0[:, :, :far])
    assert not np.array_equal(ua[:, :, far:], u0[:, :, far:])


# ------------------------------------------------ Freund's K^0 (crack) --

def test_crack_tip_sif_follows_freund_k0():
    """Suddenly loaded stationary crack (section 5.2): until waves from the
    crack mouth arrive, the mode-I stress intensity factor of a semi-infinite
    crack grows as K^0 = 2 t* sqrt(1 - 2 nu)/(1 - nu) sqrt(c_d t/pi).  On the
    1024 x 512 edge-crack plate the sqrt(t) coefficient must match within 5 %
    and the onset may lag the wave arrival by at most 40 steps."""
    from crack_sif import sif_series
    p = configs.edge_crack_plate(steps=400)
    o = Oracle(p)
    t1 = p.ny // 2          # c_d = 1 cell per step at lambda = mu
    ratio, lag = sif_series(o.step, lambda: o.moments()[3][1], p, 1e-3 * p.mu, t1)
    assert abs(ratio - 1) < 0.05, ratio
    assert 0 <= lag <= 40, lag


def test_paper_crack_follows_freund_k0():
    """Section 5.2 at the paper's own size: 400 x 400, a centred crack of
    100 cells whose faces are suddenly pushed apart (lambda/mu = 0.769).  The
    stress intensity factor at P_1, two cells ahead of a tip,
    K = sigma_xx sqrt(2 pi r), follows Freund's K^0 until the waves from the
    other tip arrive (t = l_c/c_d): fitted as c K^0(t - d) over
    [0.3, 1] l_c/c_d, c within 5 % of 1 and a delay of at most 30 steps."""
    p = configs.paper_center_crack()
    o = Oracle(p)
    par = o.lattice_params()
    cd = math.sqrt((p.lam + 2 * p.mu) / p.rho)
    cs = math.sqrt(p.mu / p.rho)
    nu = CF.nu_from_speed_ratio(cd * cd / (cs * cs))
    lc, ts = 100.0, 0.009615 * p.mu
    n_end = int(1.0 * lc / cd / par["dt_user"])
    T, K = [], []
    for n in range(0, n_end + 1, 4):
        if n:
            o.step(4)
        # P_1 lies on the crack line (between columns 199 and 200), 2 cells
        # beyond the tip at y = 249.5 (between rows 251 and 252)
        T.append(n * par["dt_user"])
        K.append(o.moments()[3][0][251:253, 199:201].mean() * math.sqrt(2 * math.pi * 2.0))
    T, K = np.array(T), np.array(K)
    sel = T >= 0.3 * lc / cd
    best = None
    for d in np.arange(0.0, 40.0, 0.5) * par["dt_user"]:
        r = np.array([CF.freund_k0(ts, nu, cd, max(t - d, 0.0)) for t in T[sel]])
        c = (K[sel] @ r) / (r @ r)
        e = np.linalg.norm(K[sel] - c * r) / np.linalg.norm(K[sel])
        if best is None or e < best[0]:
            best = (e, c, d / par["dt_user"])
    e, c, lag = best
    assert abs(c - 1) < 0.05, (c, lag, e)
    assert 0 <= lag <= 30 and e < 0.02, (c, lag, e)


def test_freund_k1_structure():
    """The evaluator of Freund's K^1 (eq:ki1) for the paper's solid: equal to
    K^0 until t = l_c/c_d, above it afterwards (the waves scattered by the
    other tip add to the opening), rising fastest at the arrival of the
    Rayleigh waves from the other tip (t = c_r l_c = 1.82 l_c/c_d) and
    levelling off after it (section 5.2)."""
    cd, cs, lc, ts = 1.0, math.sqrt(0.3611), 1.0, 1.0
    nu = CF.nu_from_speed_ratio(1 / 0.3611)
    k0 = lambda t: CF.freund_k0(ts, nu, cd, t)
    k1 = lambda t: CF.freund_k1(ts, nu, cd, cs, lc, t)
    assert k1(0.9) == k0(0.9)
    assert abs(k1(1.0 + 1e-6) - k0(1.0 + 1e-6)) < 1e-4 * k0(1.0)
    v = [k1(t) - k0(t) for t in (1.2, 1.5, 1.7, 1.8)]
    assert all(x > 0 for x in v) and v == sorted(v)
    slope_early = (k1(1.5) - k1(1.2)) / 0.3
    slope_arrival = (k1(1.85) - k1(1.75)) / 0.1
    slope_after = (k1(2.0) - k1(1.9)) / 0.1
    assert slope_arrival > 2 * slope_early
    assert slope_after < 0.5 * slope_early


def test_rayleigh_function_factors_at_zero():
    """The arctan phase g that the inner integral of eq:ki1 integrates is the
    phase of the Rayleigh function R(z) = (b^2 - 2z^2)^2 + 4 z^2 sqrt(a^2 - z^2)
    sqrt(b^2 - z^2) on its branch cut.  Its factors
    S(z) = exp(-(1/pi) int_a^b g(xi) dxi/(xi + z)) satisfy
    R = 2 (b^2 - a^2)(c_r^2 - z^2) S(z) S(-z); at z = 0 this reads
    S(0)^2 = b^4 / (2 (b^2 - a^2) c_r^2), with c_r from the Rayleigh root."""
    from scipy.integrate import quad
    for cs2 in (0.3611, 1.0 / 3.0, 0.45):
        cs = math.sqrt(cs2)
        a, b, cr = 1.0, 1.0 / cs, 1.0 / CF.rayleigh_speed(cs, 1.0)
        s0 = math.exp(-quad(lambda x: CF._freund_g(x, a, b) / x, a, b, limit=400)[0] / math.pi)
        assert abs(s0 * s0 - b ** 4 / (2 * (b * b - a * a) * cr * cr)) < 1e-9, cs2


def test_freund_constants_are_the_papers():
    """The K^1 evaluator's F_+(0) and the sampling point P_1 used by the crack
    checks are the values section 5.2 prints."""
    import inspect
    g = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))
    assert inspect.signature(CF.freund_k1).parameters["f_plus0"].default == g["freund_F_plus_0"]["value"]
    assert inspect.signature(CF.freund_k1_curve).parameters["f_plus0"].default == g["freund_F_plus_0"]["value"]
    # P_1 two cells ahead of the upper tip: 0.52 l_c from the centre, the tip at 0.5 l_c, dx = l_c/100
    p1 = g["crack_point_P1"]
    assert abs((p1["y_over_lc"] - 0.5) * p1["crack_length_cells"] - 2.0) < 1e-12 and p1["x_over_lc"] == 0.0


def _k1_integral_by_contour(T, a, b, cr, eps=2e-5, delta=1e-4):
    """The integral of eq:ki1 evaluated as printed, in complex arithmetic:
    principal square roots, the arctan continued off the real axis as
    (log(D + iN) - log(D - iN))/2i, the inner pole at xi = eta passed on a
    semicircle of radius eps above the real axis (quadrature in the angle),
    and the outer pole at eta = c_r excluded symmetrically (principal
    value).  Shares nothing with closed_forms but the Rayleigh root."""
    from scipy.integrate import quad

    def gc(xi):
        N = 4 * xi * xi * np.sqrt((xi * xi - a * a) * (b * b - xi * xi) + 0j)
        D = (b * b - 2 * xi * xi) ** 2 + 0j
        return (np.log(D + 1j * N) - np.log(D - 1j * N)) / 2j

    def inner(eta):
        f = lambda xi: (gc(xi) * 2 * eta / (xi * xi - eta * eta)).real
        if not a < eta < b:
            return quad(f, a, b, limit=400)[0] + 0j
        s = quad(f, a, eta - eps, limit=400)[0] + quad(f, eta + eps, b, limit=400)[0]
        z = lambda th: eta + eps * np.exp(1j * th)
        arc = lambda th: gc(z(th)) * 2 * eta / (z(th) ** 2 - eta * eta) * 1j * eps * np.exp(1j * th)
        # the semicircle runs from theta = pi down to 0
        return s - (quad(lambda th: arc(th).real, 0, math.pi)[0] + 1j * quad(lambda th: arc(th).imag, 0, math.pi)[0])

    def h(eta):
        return (np.sqrt(T - eta + 0j) * np.sqrt((a - eta) / (a + eta) + 0j) * (cr + eta) / (cr - eta) / eta
                * np.exp(inner(eta) / math.pi)).imag

    if T <= cr:
        return quad(h, a, T, limit=200)[0]
    return quad(h, a, cr - delta, limit=200)[0] + quad(h, cr + delta, T, limit=200)[0]


def test_freund_k1_matches_contour_evaluation():
    """The real form the K^1 evaluator integrates (principal values plus the
    phase that the semicircle around the inner pole contributes) equals
    eq:ki1 evaluated literally along the contour the paper describes, before
    and after the Rayleigh pole.  Dropping the semicircle's contribution
    makes the first value 8 times larger."""
    cs = math.sqrt(0.3611)
    a, b, cr = 1.0, 1.0 / cs, 1.0 / CF.rayleigh_speed(cs, 1.0)
    for T, tol in ((1.5, 1e-6), (1.95, 1e-3)):
        lit = _k1_integral_by_contour(T, a, b, cr)
        red = CF._freund_outer(T, a, b, cr, lambda e: CF._freund_inner(e, a, b))
        assert abs(lit - red) <= tol * abs(red), (T, lit, red)
    curve = CF.freund_k1_curve(1.0, CF.nu_from_speed_ratio(1 / 0.3611), 1.0, cs, 1.0, [1.3, 1.9])
    for t, v in zip((1.3, 1.9), curve):
        assert abs(v - CF.freund_k1(1.0, CF.nu_from_speed_ratio(1 / 0.3611), 1.0, cs, 1.0, t)) < 1e-5 * v


def test_paper_crack_follows_freund_k1():
    """Section 5.2 past the first scattered waves: on the paper's 400 x 400
    crack, from t = l_c/c_d (when the waves scattered by the other tip
    arrive) to 1.75 l_c/c_d, the stress intensity factor at P_1 keeps the
    ratio to Freund's K^1 that it has at l_c/c_d, within 2 % (the K^0
    continuation drifts by 5 %); its steepest rise comes with the Rayleigh
    waves from the other tip, at c_r l_c within 0.05 l_c/c_d."""
    from crack_sif import paper_crack_k1_window
    p = configs.paper_center_crack()
    o = Oracle(p)
    _, _, drift, t_steep, t_rayleigh = paper_crack_k1_window(o.step, lambda: o.moments()[3][0], p)
    assert drift < 0.02, drift
    assert abs(t_steep - t_rayleigh) < 0.05, (t_steep, t_rayleigh)