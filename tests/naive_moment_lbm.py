"""A second, deliberately naive formulation of the same solid-LBM step, used
only to cross-check the CPU reference on tiny grids.

Differences from the reference, on purpose:

* sites are a dict keyed by (ix, iy) holding plain Python lists;
* the collision is done in moment space: populations are mapped to the nine
  moments (rho, j, P, the two third-order moments and the fourth-order one)
  with the matrix of monomials of the lattice velocities, every moment is
  relaxed toward its equilibrium value, and the result is mapped back.  The
  equilibrium moments are the values the paper's equilibrium (eq:fieq) must
  have -- rho, j, P, c_s^2 j for the third-order pair and
  (P_xx + P_yy)/3 - rho/9 for the fourth-order moment -- worked out by hand
  rather than evaluated from the population formula;
* the boundary rules are written with the paper's link length l_i and wall
  distance s_i instead of the fraction q.
"""
import math

import numpy as np

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
WGT = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
CS2 = 1.0 / 3.0


def _basis(i):
    cx, cy = CX[i], CY[i]
    return [1, cx, cy, cx * cx, cy * cy, cx * cy, cx * cy * cy, cx * cx * cy, cx * cx * cy * cy]


M = np.array([[_basis(i)[a] for i in range(9)] for a in range(9)], dtype=float)
MINV = np.linalg.inv(M)


class NaiveLBM:
    def __init__(self, plate):
        p = plate
        self.p = p
        self.nx, self.ny = p.nx, p.ny
        s_sigma = 3.0 * p.mu
        self.dt = math.sqrt(p.rho / (3.0 * p.mu))
        self.s_v = 1.0 / self.dt
        self.lam = p.lam / s_sigma
        self.mu = p.mu / s_sigma
        self.tau = p.tau
        self.F = (p.force[0] / s_sigma, p.force[1] / s_sigma)
        self.groups = []
        for g in p.groups:
            scale = self.s_v if g.kind == 1 else s_sigma
            ramp = g.ramp_time / self.dt if g.profile == 1 else None
            self.groups.append((g.kind, (g.value[0] / scale, g.value[1] / scale), ramp))
        self.sites = {}
        for iy in range(p.ny):
            for ix in range(p.nx):
                if p.mask[iy, ix]:
                    self.sites[(ix, iy)] = None
        self.cut = {}
        for L in p.links:
            s = int(L["site"])
            key = ((s % p.nx, s // p.nx), int(L["dir"]))
            self.cut[key] = (float(L["q"]), int(L["group"]), int(L["group2"]),
                             tuple(L["normal"]), tuple(L["normal2"]))
        self.t = 0

    def wrap(self, ix, iy):
        if self.p.periodic_x:
            ix %= self.nx
        if self.p.periodic_y:
            iy %= self.ny
        return ix, iy

    def set_f(self, f):
        for (ix, iy) in self.sites:
            self.sites[(ix, iy)] = [float(f[i, iy, ix]) for i in range(9)]

    def get_f(self):
        out = np.zeros((9, self.ny, self.nx))
        for (ix, iy), v in self.sites.items():
            out[:, iy, ix] = v
        return out

    def _amp(self, g):
        ramp = self.groups[g][2]
        return 1.0 if ramp is None else min(self.t / ramp, 1.0)

    def step(self):
        mom = {}
        for key, f in self.sites.items():
            mom[key] = M @ np.array(f)
        rho = {k: m[0] for k, m in mom.items()}
        new = {k: [None] * 9 for k in self.sites}
        fcol = {}
        for (ix, iy), m in mom.items():
            # density gradient across the eight neighbours
            g = [0.0, 0.0]
            for i in range(1, 9):
                if ((ix, iy), i) not in self.cut:
                    r = rho[self.wrap(ix + CX[i], iy + CY[i])]
                elif ((ix, iy), OPP[i]) not in self.cut:
                    r = 2 * rho[(ix, iy)] - rho[self.wrap(ix - CX[i], iy - CY[i])]
                else:
                    r = rho[(ix, iy)]
                g[0] += WGT[i] * CX[i] * r / CS2
                g[1] += WGT[i] * CY[i] * r / CS2
            r0 = m[0]
            S = [self.F[a] + (self.mu - self.lam) / r0 * g[a] for a in range(2)]
            jx, jy = m[1] + S[0] / 2, m[2] + S[1] / 2
            pxx, pyy, pxy = m[3], m[4], m[5]
            meq = np.array([r0, jx, jy, pxx, pyy, pxy, CS2 * jx, CS2 * jy, (pxx + pyy) / 3 - r0 / 9])
            mpsi = np.array([0, S[0], S[1], 0, 0, 0, CS2 * S[0], CS2 * S[1], 0])
            mc = m - (m - meq) / self.tau + (1 - 1 / (2 * self.tau)) * mpsi
            fcol[(ix, iy)] = list(MINV @ mc)
        for (ix, iy), fc in fcol.items():
            new[(ix, iy)][0] = fc[0]
            for i in range(1, 9):
                if ((ix, iy), i) not in self.cut:
                    new[self.wrap(ix + CX[i], iy + CY[i])][i] = fc[i]
        for ((ix, iy), k), (q, g1, g2, n1, n2) in self.cut.items():
            kb = OPP[k]
            l = math.hypot(CX[k], CY[k])
            s = q * l
            behind = ((ix, iy), kb) not in self.cut
            y = self.wrap(ix - CX[k], iy - CY[k])
            if behind:
                a = (l - 2 * s) / (l + 2 * s)
                b = 2 * l / (l + 2 * s)
            else:
                a, b = 0.0, 1.0
            fk = fcol[(ix, iy)][k]
            fkb = fcol[(ix, iy)][kb]
            fky = fcol[y][k] if behind else 0.0
            kinds = [self.groups[g1][0]] + ([self.groups[g2][0]] if g2 >= 0 else [])
            if 1 in kinds:
                gd = g1 if self.groups[g1][0] == 1 else g2
                v = self.groups[gd][1]
                am = self._amp(gd)
                js = (rho[(ix, iy)] * v[0] * am, rho[(ix, iy)] * v[1] * am)
                val = fk + a * (fky - fkb) - b * 2 / CS2 * WGT[k] * (CX[k] * js[0] + CY[k] * js[1])
            else:
                use_y = behind and self.p.neumann_order == 1
                rx = rho[(ix, iy)]
                rbd = ((l + s) / l * rx - s / l * rho[y]) if use_y else rx

                def cauchy(site):
                    mm = mom[site]
                    d = (self.lam - self.mu) * (1 - mm[0])
                    return np.array([[-mm[3] + d, -mm[5]], [-mm[5], -mm[4] + d]])
                if g2 >= 0:
                    tA = np.array(self.groups[g1][1]) * self._amp(g1)
                    tB = np.array(self.groups[g2][1]) * self._amp(g2)
                    sig = np.outer(tA, n1) + np.outer(tB, n2)
                    sig = (sig + sig.T) / 2
                else:
                    t = np.array(self.groups[g1][1]) * self._amp(g1)
                    # rotation with rows e_n, e_t (eq:trafocauchy)
                    T = np.array([[n1[0], n1[1]], [-n1[1], n1[0]]])
                    sn = T @ cauchy((ix, iy)) @ T.T
                    stt = sn[1, 1]
                    if use_y:
                        stt = (l + s) / l * stt - s / l * (T @ cauchy(y) @ T.T)[1, 1]
                    tn = T @ t
                    sig_n = np.array([[tn[0], tn[1]], [tn[1], stt]])
                    sig = T.T @ sig_n @ T
                Pst = -sig + (self.lam - self.mu) * (1 - rbd) * np.eye(2)
                c = np.array([CX[k], CY[k]], dtype=float)
                sec = np.sum((Pst - rbd * CS2 * np.eye(2)) * (np.outer(c, c) - CS2 * np.eye(2)))
                E = 2 * WGT[k] * (rbd + sec / (2 * CS2 * CS2))
                val = -fk - a * (fky + fkb) + b * E
            new[(ix, iy)][kb] = val
        for k, v in new.items():
            assert all(x is not None for x in v), k
        self.sites = new
        self.t += 1
