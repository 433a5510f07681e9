"""Brute-force loop form of one D3Q19 step of the solid lattice-Boltzmann
method (test helper): explicit per-site loops and neighbour indices, written
from the definitions (eq:moments, eq:sourceterm, eq:fieq, eq:coll,
eq:stream, eq:bbcon and eq:abbcon, or eq:bbnoncon and eq:abbnoncon for walls
at q != 1/2, with rho_bd and the tangential stress at the site or
extrapolated along the link) without sharing code with the reference it
checks.  Lattice units inside; the box in user units."""
import itertools
import math

import numpy as np

DIRICHLET, NEUMANN = 1, 2


def _w(c):
    return {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[sum(a * a for a in c)]


def _feq(c, rho, j, P):
    cs2 = 1.0 / 3.0
    v = rho + sum(c[a] * j[a] for a in range(3)) / cs2
    v += sum((P[a][b] - cs2 * rho * (a == b)) * (c[a] * c[b] - cs2 * (a == b))
             for a in range(3) for b in range(3)) / (2 * cs2 * cs2)
    return _w(c) * v


def _factor(w, step, dt_user):
    """A wall's or group's time profile at step `step`: 1, or min(t / ramp_time, 1)
    with t = step dt_user (RAMP, profile 1)."""
    if getattr(w, "profile", 0) == 1:
        return min(step * dt_user / w.ramp_time, 1.0)
    return 1.0


def naive_step(box, f, U, order, step=0):
    """f [19, nz, ny, nx] in the direction order `order` (tuples), U [3, ...]:
    returns (f, U) after one step from step index `step` (the time of the
    boundary values)."""
    nz, ny, nx = f.shape[1:]
    vel = list(itertools.product((-1, 0, 1), repeat=3))
    vel = [c for c in vel if sum(a * a for a in c) <= 2]
    assert sorted(vel) == sorted(order)
    idx = {c: k for k, c in enumerate(order)}
    s_sigma = 3 * box.mu
    s_v = math.sqrt(3 * box.mu / box.rho)
    lamL, muL = box.lam / s_sigma, box.mu / s_sigma
    F = [a / s_sigma for a in box.force]
    walls = box.x_walls
    tau = box.tau
    mask = box.mask
    links = {}
    if mask is not None:
        for L in box.links:
            s_ = int(L["site"])
            links[(s_ % (ny * nx) % nx, s_ % (ny * nx) // nx, s_ // (ny * nx), order[int(L["dir"])])] = L

    def inside_x(x):
        return walls is None or 0 <= x < nx

    def material(x, y, z):
        if not inside_x(x):
            return False
        if mask is None:
            return True
        xx, yy, zz = wrap(x, y, z)
        return bool(mask[zz, yy, xx])

    def wrap(x, y, z):
        return (x % nx, y % ny, z % nz)

    def open_link(x, y, z, c):
        """The link from material site (x, y, z) along c reaches material
        without crossing a wall, a cavity's wall or a crack."""
        if not material(x + c[0], y + c[1], z + c[2]):
            return False
        return mask is None or (x, y, z, c) not in links

    rho = np.zeros((nz, ny, nx))
    J = np.zeros((3, nz, ny, nx))
    PP = np.zeros((3, 3, nz, ny, nx))
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        for c in vel:
            v = f[idx[c], z, y, x]
            rho[z, y, x] += v
            for a in range(3):
                J[a, z, y, x] += v * c[a]
                for b in range(3):
                    PP[a, b, z, y, x] += v * c[a] * c[b]

    fcol = np.zeros_like(f)
    Un = U.copy()
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if not material(x, y, z):
            continue
        r = rho[z, y, x]
        grad = [0.0, 0.0, 0.0]
        for c in vel:
            if c == (0, 0, 0):
                continue
            cb = tuple(-a for a in c)
            if open_link(x, y, z, c):
                xx, yy, zz = wrap(x + c[0], y + c[1], z + c[2])
                rn = rho[zz, yy, xx]
            elif open_link(x, y, z, cb):
                xx, yy, zz = wrap(x - c[0], y - c[1], z - c[2])
                rn = 2 * r - rho[zz, yy, xx]
            else:
                rn = r
            for a in range(3):
                grad[a] += 3 * _w(c) * c[a] * rn
        S = [F[a] + (muL - lamL) / r * grad[a] for a in range(3)]
        j = [J[a, z, y, x] + S[a] / 2 for a in range(3)]
        P = [[PP[a, b, z, y, x] for b in range(3)] for a in range(3)]
        for c in vel:
            fi = f[idx[c], z, y, x]
            psi = 3 * _w(c) * sum(c[a] * S[a] for a in range(3))
            fcol[idx[c], z, y, x] = fi - (fi - _feq(c, r, j, P)) / tau + (1 - 1 / (2 * tau)) * psi
        for a in range(3):
            Un[a, z, y, x] += j[a] / r

    fnew = np.zeros_like(f)
    if mask is not None:
        rest = [_feq(c, 1.0, [0.0, 0.0, 0.0], [[0.0] * 3 for _ in range(3)]) for c in order]
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            if not mask[z, y, x]:
                fnew[:, z, y, x] = rest
                Un[:, z, y, x] = 0.0
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if not material(x, y, z):
            continue
        for c in vel:
            if open_link(x, y, z, c):
                xx, yy, zz = wrap(x + c[0], y + c[1], z + c[2])
                fnew[idx[c], zz, yy, xx] = fcol[idx[c], z, y, x]
                continue
            if mask is not None:
                fnew[idx[tuple(-a for a in c)], z, y, x] = _cut_link(box, fcol, idx, vel, links[(x, y, z, c)],
                                                                     x, y, z, c, open_link, wrap, lamL, muL,
                                                                     s_v, s_sigma, step)
                continue
            # the link leaves through a wall: the population returns to x
            side = 0 if x + c[0] < 0 else 1
            kind, q = walls[side].kind, walls[side].q
            a_t = _factor(walls[side], step, math.sqrt(box.rho / (3 * box.mu)))
            value = [v * a_t for v in walls[side].value]
            cb = tuple(-a for a in c)
            fc = fcol[idx[c], z, y, x]
            fcb = fcol[idx[cb], z, y, x]
            r = sum(fcol[idx[d], z, y, x] for d in vel)
            Pm = [[sum(fcol[idx[d], z, y, x] * d[a] * d[b] for d in vel) for b in range(3)] for a in range(3)]
            # the site behind x along the link, x - c (inside when nx > 1)
            has_b = nx > 1
            if has_b:
                bx, by, bz = wrap(x - c[0], y - c[1], z - c[2])
                fb = fcol[idx[c], bz, by, bx]
                rb = sum(fcol[idx[d], bz, by, bx] for d in vel)
                Pb = [[sum(fcol[idx[d], bz, by, bx] * d[a] * d[b] for d in vel) for b in range(3)] for a in range(3)]
                kap, bet = (1 - 2 * q) / (1 + 2 * q), 2 / (1 + 2 * q)
            else:
                fb, kap, bet = 0.0, 0.0, 1.0
            if kind == DIRICHLET:
                vL = [v / s_v for v in value]
                fnew[idx[cb], z, y, x] = (fc + kap * (fb - fcb)
                                          - bet * 6 * _w(c) * sum(c[a] * r * vL[a] for a in range(3)))
            else:
                t = [v / s_sigma for v in value]
                n = [-1.0 if side == 0 else 1.0, 0.0, 0.0]

                def cauchy(rr, PP_):
                    return [[-PP_[a][b] + (lamL - muL) * (1 - rr) * (a == b) for b in range(3)] for a in range(3)]

                sig = cauchy(r, Pm)
                rbd = r
                if has_b and box.neumann_order == 1:
                    sb = cauchy(rb, Pb)
                    sig = [[(1 + q) * sig[a][b] - q * sb[a][b] for b in range(3)] for a in range(3)]
                    rbd = (1 + q) * r - q * rb
                # boundary stress: normal part from the traction, tangential
                # block (rows and columns y, z) from the site or extrapolated
                st = [[0.0] * 3 for _ in range(3)]
                for a in (1, 2):
                    for b in (1, 2):
                        st[a][b] = sig[a][b]
                for a in range(3):
                    st[a][0] = t[a] * n[0]
                    st[0][a] = t[a] * n[0]
                Ps = [[-st[a][b] + (lamL - muL) * (1 - rbd) * (a == b) for b in range(3)] for a in range(3)]
                fnew[idx[cb], z, y, x] = -fc - kap * (fb + fcb) + bet * 2 * _feq(c, rbd, [0.0, 0.0, 0.0], Ps)
    return fnew, Un


def _cut_link(box, fcol, idx, vel, L, x, y, z, c, open_link, wrap, lamL, muL, s_v, s_sigma, step=0):
    """The population returning to material site (x, y, z) along the cut link
    in direction c, with the link's own q, outward normal and group."""
    q = float(L["q"])
    n = [float(v) for v in L["normal"]]
    G = box.groups[int(L["group"])]
    g2 = int(L["group2"]) if "group2" in L.dtype.names else -1
    G2 = box.groups[g2] if g2 >= 0 else None
    if G.kind != DIRICHLET and G2 is not None and G2.kind == DIRICHLET:
        G = G2                       # an edge of a Dirichlet and a Neumann face: Dirichlet
    cb = tuple(-a for a in c)
    fc = fcol[idx[c], z, y, x]
    fcb = fcol[idx[cb], z, y, x]

    def mom(xx, yy, zz):
        r = sum(fcol[idx[d], zz, yy, xx] for d in vel)
        Pm = [[sum(fcol[idx[d], zz, yy, xx] * d[a] * d[b] for d in vel) for b in range(3)] for a in range(3)]
        return r, Pm

    r, Pm = mom(x, y, z)
    # no site behind x when the opposite link is cut as well
    has_b = open_link(x, y, z, cb)
    if has_b:
        bx, by, bz = wrap(x - c[0], y - c[1], z - c[2])
        fb = fcol[idx[c], bz, by, bx]
        kap, bet = (1 - 2 * q) / (1 + 2 * q), 2 / (1 + 2 * q)
    else:
        fb, kap, bet = 0.0, 0.0, 1.0
    if G.kind == DIRICHLET:
        vL = [v / s_v * _factor(G, step, 1 / s_v) for v in G.value]
        return fc + kap * (fb - fcb) - bet * 6 * _w(c) * sum(c[a] * r * vL[a] for a in range(3))

    def cauchy(rr, PP_):
        return [[-PP_[a][b] + (lamL - muL) * (1 - rr) * (a == b) for b in range(3)] for a in range(3)]

    sig = cauchy(r, Pm)
    rbd = r
    if has_b and box.neumann_order == 1:
        rb, Pb = mom(bx, by, bz)
        sb = cauchy(rb, Pb)
        sig = [[(1 + q) * sig[a][b] - q * sb[a][b] for b in range(3)] for a in range(3)]
        rbd = (1 + q) * r - q * rb
    aG = _factor(G, step, 1 / s_v)
    t = [(G.value[a] / s_sigma - G.pressure / s_sigma * n[a]) * aG for a in range(3)]
    if G2 is None:
        tn = sum(t[a] * n[a] for a in range(3))
        Pi = [[(a == b) - n[a] * n[b] for b in range(3)] for a in range(3)]
        st = [[sum(Pi[a][e] * sig[e][f] * Pi[f][b] for e in range(3) for f in range(3))
               + n[a] * t[b] + t[a] * n[b] - tn * n[a] * n[b] for b in range(3)] for a in range(3)]
    else:
        # an edge of two Neumann faces: in the basis (n, n2, e = n x n2), the
        # rows of n and n2 from the tractions (their shear averaged), the
        # edge component from the material
        n2 = [float(v) for v in L["normal2"]]
        aG2 = _factor(G2, step, 1 / s_v)
        t2 = [(G2.value[a] / s_sigma - G2.pressure / s_sigma * n2[a]) * aG2 for a in range(3)]
        e = [n[1] * n2[2] - n[2] * n2[1], n[2] * n2[0] - n[0] * n2[2], n[0] * n2[1] - n[1] * n2[0]]
        d = lambda u, v: sum(u[a] * v[a] for a in range(3))
        basis = [n, n2, e]
        comp = [[d(t, n), (d(t, n2) + d(t2, n)) / 2, d(t, e)],
                [(d(t, n2) + d(t2, n)) / 2, d(t2, n2), d(t2, e)],
                [d(t, e), d(t2, e), sum(e[a] * sig[a][b] * e[b] for a in range(3) for b in range(3))]]
        st = [[sum(comp[i][j] * basis[i][a] * basis[j][b] for i in range(3) for j in range(3)) for b in range(3)]
              for a in range(3)]
    Ps = [[-st[a][b] + (lamL - muL) * (1 - rbd) * (a == b) for b in range(3)] for a in range(3)]
    return -fc - kap * (fb + fcb) + bet * 2 * _feq(c, rbd, [0.0, 0.0, 0.0], Ps)
