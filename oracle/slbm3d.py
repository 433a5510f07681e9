"""Plain CPU reference of a three-dimensional (D3Q19) form of the solid
lattice-Boltzmann step (TEST INFRASTRUCTURE).

Only the test suite and the benchmark's CPU-baseline leg use this module.  It
shares no code with the HIP library and is never a fallback for it.

The paper (Faust, Schlueter, H. Mueller, R. Mueller, 2022) treats plane
strain on D2Q9 and notes that its boundary rules generalise to three
dimensions (section 1).  This module takes every step of the two-dimensional
method in the paper's order, on the D3Q19 lattice (same c_s^2 = 1/3, weights
1/3, 1/18, 1/36, fourth-order isotropic like D2Q9), in float64 numpy:

  moments (eq:moments) -> source term S = F + (mu - lambda)/rho grad(rho)
  (eq:sourceterm) -> equilibrium with the populations' own second moment
  (eq:fieq) -> BGK collision with forcing (eq:coll) -> displacement
  integration U += j/rho -> streaming along uncut links (eq:stream) ->
  boundary rules on the links cut by the walls (eq:bbcon for Dirichlet,
  eq:abbcon for Neumann).

Readings beyond the paper (the three-dimensional extension):

* Walls are lattice-conforming planes at x = -1/2 and x = nx - 1/2 (q = 1/2
  on every cut link, so the rules' interpolation terms vanish); y and z are
  periodic.
* The Neumann rule's boundary Cauchy stress is
      sigma* = Pi sigma(x) Pi + n (x) t* + t* (x) n - (t*.n) n (x) n,
  Pi = I - n n: its normal part is fixed by the traction t* (sigma*.n = t*),
  its tangential block taken at the boundary site (the rule with the
  boundary-site values, the stable one of the two the workloads use).  In two
  dimensions this is the paper's eq:trafocauchy with sigma_tt at the site.
* The density gradient uses the isotropic D3Q19 stencil,
  grad(rho) = 3 sum_i w_i c_i rho(x + c_i), with the neighbour across a cut
  link extrapolated as 2 rho(x) - rho(x - c_i) (rho(x) if that link is cut
  too), as in two dimensions.

Units: user units in and out, dx = 1 cell; lattice units inside with
dx = dt = 1, rho0 = 1, c_s^2 = 1/3, so dt_user = sqrt(rho/(3 mu)).

Precision: float64, or with ``extended=True`` the x87 80-bit long double
(numpy.longdouble) for every array and constant.  The reference works on the
unshifted populations, of order one, so in float64 the small deviations it
computes (momentum, stress, displacement) carry relative rounding near 1e-12;
the extended form is the reference for float64 parity at that level.
"""
from __future__ import annotations

import numpy as np

DIRICHLET = 1
NEUMANN = 2
STEP = 0
RAMP = 1

# D3Q19: rest, the six axis links, the twelve face diagonals
C = np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
Q = len(C)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
OPP = np.array([int(np.flatnonzero((C == -c).all(1))[0]) for c in C])
CS2 = 1.0 / 3.0


def _lattice_constants(dtype):
    """Weights and c_s^2 formed in `dtype`."""
    one = dtype(1)
    w = np.array([one / 3] + [one / 18] * 6 + [one / 36] * 12, dtype=dtype)
    return w, one / 3
# symmetric-tensor components in the order xx, yy, zz, xy, xz, yz
SYM = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def sym_to_full(p6):
    """[6, ...] -> [3, 3, ...]"""
    m = np.empty((3, 3) + p6.shape[1:])
    for k, (a, b) in enumerate(SYM):
        m[a, b] = p6[k]
        m[b, a] = p6[k]
    return m


def full_to_sym(m):
    return np.stack([m[a, b] for a, b in SYM])


def equilibrium(rho, j, P):
    """eq:fieq on D3Q19: f_eq,i = w_i [rho + c_i.j / c_s^2
    + (P - c_s^2 rho I):(c_i c_i - c_s^2 I) / (2 c_s^4)].
    rho [...], j [3, ...], P [3, 3, ...] -> [19, ...], in rho's precision."""
    rho = np.asarray(rho)
    W, CS2 = _lattice_constants(rho.dtype.type if rho.dtype == np.longdouble else np.float64)
    out = np.empty((Q,) + np.shape(rho), dtype=rho.dtype if rho.dtype == np.longdouble else np.float64)
    for i in range(Q):
        c = C[i]
        cj = c[0] * j[0] + c[1] * j[1] + c[2] * j[2]
        pc = 0.0
        for a in range(3):
            for b in range(3):
                pc = pc + (P[a, b] - CS2 * rho * (a == b)) * (c[a] * c[b] - CS2 * (a == b))
        out[i] = W[i] * (rho + cj / CS2 + pc / (2.0 * CS2 * CS2))
    return out


class Oracle3D:
    """One box advanced by the reference.  ``box`` is a
    :class:`slbm_workloads.box3d.Box3`."""

    def __init__(self, box, extended: bool = False):
        b = box
        self.dt = np.longdouble if extended else np.float64
        self.W, self.cs2 = _lattice_constants(self.dt)
        if not (b.mu > 0 and b.rho > 0):
            raise ValueError("mu and rho must be positive")
        if not b.tau > 0.5:
            raise ValueError("tau must exceed 1/2")
        self.box = b
        self.shape = (b.nz, b.ny, b.nx)
        # unit mapping (section 5.1): c_s = sqrt(mu/rho) = dx/(sqrt(3) dt)
        self.dt_user = np.sqrt(b.rho / (3.0 * b.mu))
        self.s_sigma = 3.0 * b.mu
        self.s_v = 1.0 / self.dt_user
        self.mu = self.dt(b.mu) / self.dt(self.s_sigma)
        self.lam = self.dt(b.lam) / self.dt(self.s_sigma)
        self.tau = self.dt(b.tau)
        self.F = np.array(b.force, dtype=self.dt) / self.dt(self.s_sigma)
        self.walls = None
        if b.neumann_order not in (0, 1):
            raise ValueError("neumann_order must be 0 or 1")
        self.norder = b.neumann_order
        if b.x_walls is not None:
            self.walls = []
            for wall in b.x_walls:
                if wall.kind not in (DIRICHLET, NEUMANN):
                    raise ValueError("wall kind must be Dirichlet or Neumann")
                if not 0.0 < wall.q <= 1.0:
                    raise ValueError("wall q must be in (0, 1]")
                scale = self.s_v if wall.kind == DIRICHLET else self.s_sigma
                self.walls.append((wall.kind, np.array(wall.value, dtype=self.dt) / self.dt(scale),
                                   self.dt(wall.q)))
            self.wprof = [self._profile_of(w) for w in b.x_walls]
        # cut[i] marks the sites whose link i leaves the material through a wall
        self.cut = np.zeros((Q,) + self.shape, dtype=bool)
        if self.walls is not None:
            for i in range(Q):
                if C[i, 0] < 0:
                    self.cut[i, :, :, 0] = True
                elif C[i, 0] > 0:
                    self.cut[i, :, :, -1] = True
        self.mask = None
        if b.mask is not None:
            self._general(b)
        self.f = np.repeat(equilibrium(np.ones(1, dtype=self.dt), np.zeros((3, 1), dtype=self.dt),
                                       np.zeros((3, 3, 1), dtype=self.dt)), b.n_sites, 1)
        self.f = self.f.reshape((Q,) + self.shape)
        self.rest = self.f[:, :1, :1, :1].copy()
        self.U = np.zeros((3,) + self.shape, dtype=self.dt)
        self.n = 0

    def _general(self, b):
        """A box with cut links (periodic on every axis): the material mask,
        the links, their groups in lattice units.  A cut link ends in the void
        (a cavity's wall), or in the material across a crack: then the link
        back from the far site must be listed too (the crack's other face)."""
        if b.x_walls is not None:
            raise ValueError("a box with a material mask is periodic on every axis")
        mask = np.asarray(b.mask).astype(bool)
        if mask.shape != self.shape:
            raise ValueError("mask shape must be (nz, ny, nx)")
        self.mask = mask
        L = b.links
        site = L["site"].astype(np.int64)
        k = L["dir"].astype(np.int64)
        if ((site < 0) | (site >= mask.size)).any():
            raise ValueError("a cut link's site is out of range")
        if ((k < 1) | (k >= Q)).any():
            raise ValueError("a cut link's direction must be one of the 18 moving ones")
        z, rem = np.divmod(site, b.ny * b.nx)
        y, x = np.divmod(rem, b.nx)
        if not mask[z, y, x].all():
            raise ValueError("a cut link starts at a void site")
        fz, fy, fx = (z + C[k, 2]) % b.nz, (y + C[k, 1]) % b.ny, (x + C[k, 0]) % b.nx
        q = L["q"]
        if not ((q > 0) & (q <= 1)).all():
            raise ValueError("q must be in (0, 1]")
        n = np.asarray(L["normal"], dtype=float).reshape(-1, 3)
        if (np.abs(np.linalg.norm(n, axis=1) - 1) > 1e-9).any():
            raise ValueError("normals must be unit vectors")
        g = L["group"].astype(np.int64)
        has2 = "group2" in L.dtype.names
        g2 = L["group2"].astype(np.int64) if has2 else np.full(len(site), -1)
        n2 = np.asarray(L["normal2"], dtype=float) if has2 else np.zeros((len(site), 3))
        ng = len(b.groups)
        if ((g < 0) | (g >= ng)).any() or ((g2 < -1) | (g2 >= ng)).any():
            raise ValueError("a cut link's group is out of range")
        two = g2 >= 0
        if two.any():
            if (np.abs(np.linalg.norm(n2[two], axis=1) - 1) > 1e-9).any():
                raise ValueError("second normals must be unit vectors")
            if (np.abs(np.einsum("ma,ma->m", n[two], n2[two])) > 1e-9).any():
                raise ValueError("a link through an edge needs orthogonal normals")
        if len(set(zip(site.tolist(), k.tolist()))) != len(site):
            raise ValueError("a cut link is listed twice")
        self.cut[k, z, y, x] = True
        # a link into the material crosses a crack: both faces list their link
        crack = mask[fz, fy, fx]
        if not self.cut[OPP[k[crack]], fz[crack], fy[crack], fx[crack]].all():
            raise ValueError("a cut link into the material needs the link back (the crack's other face)")
        # every link from the material into the void must be listed
        for i in range(1, Q):
            far_void = ~np.roll(mask, (-C[i, 2], -C[i, 1], -C[i, 0]), axis=(0, 1, 2))
            if (far_void & mask & ~self.cut[i]).any():
                raise ValueError("a link from the material into the void is not listed")
        self.links = dict(z=z, y=y, x=x, k=k, q=q.astype(self.dt), g=g, n=n.astype(self.dt), g2=g2,
                          n2=n2.astype(self.dt))
        self.gkind = np.array([g.kind for g in b.groups])
        self.gprof = [self._profile_of(g) for g in b.groups]
        self.gval = []
        for g in b.groups:
            if g.kind not in (DIRICHLET, NEUMANN):
                raise ValueError("group kind must be Dirichlet or Neumann")
            scale = self.s_v if g.kind == DIRICHLET else self.s_sigma
            self.gval.append((np.array(g.value, dtype=self.dt) / self.dt(scale),
                              self.dt(getattr(g, "pressure", 0.0)) / self.dt(self.s_sigma)))

    def _profile_of(self, w):
        """(profile, ramp length in steps) of a wall or group."""
        prof = getattr(w, "profile", STEP)
        if prof == STEP:
            return (STEP, self.dt(1))
        if prof != RAMP or not getattr(w, "ramp_time", 0.0) > 0:
            raise ValueError("a profile is STEP, or RAMP with a positive ramp time")
        return (RAMP, self.dt(w.ramp_time) / self.dt(self.dt_user))

    def _factor(self, prof):
        """The profile's factor at the current step n (the rule applied to the
        post-collision state of step n takes the value at t_n = n dt)."""
        kind, T = prof
        return self.dt(1) if kind == STEP else min(self.dt(self.n) / T, self.dt(1))

    # -------------------------------------------------------------- steps
    def _moments(self, f):
        c = C.astype(self.dt)
        rho = f.sum(0)
        j = np.einsum("ia,i...->a...", c, f)
        P = np.einsum("ia,ib,i...->ab...", c, c, f)
        return rho, j, P

    def _neighbour(self, a, i, sign):
        """a(x + sign c_i) with wrap on the periodic axes (x only if periodic;
        callers do not read across a wall)."""
        c = C[i] * sign
        return np.roll(a, (-c[2], -c[1], -c[0]), axis=(0, 1, 2))

    def _source(self, rho):
        """eq:sourceterm, S = F + ((mu - lambda)/rho) grad(rho), isotropic
        stencil; across a cut link the neighbour is 2 rho(x) - rho(x - c_i),
        or rho(x) if the opposite link is cut too."""
        grad = np.zeros((3,) + self.shape, dtype=self.dt)
        for i in range(1, Q):
            r = self._neighbour(rho, i, +1)
            if self.walls is not None or self.mask is not None:
                ext = np.where(self.cut[OPP[i]], rho, 2.0 * rho - self._neighbour(rho, i, -1))
                r = np.where(self.cut[i], ext, r)
            for a in range(3):
                if C[i, a]:
                    grad[a] += self.W[i] * C[i, a] * r
        grad /= self.cs2
        S = self.F[:, None, None, None] + ((self.mu - self.lam) / rho) * grad
        return S

    def _cauchy(self, rho, P):
        """sigma = -P + (lambda - mu)(1 - rho) I (eq:poissonstress with
        eq:approxdiv), lattice units, [3, 3, ...]."""
        s = -P.copy()
        for a in range(3):
            s[a, a] += (self.lam - self.mu) * (1.0 - rho)
        return s

    def step(self, nsteps=1):
        for _ in range(int(nsteps)):
            f = self.f
            rho, j, P = self._moments(f)
            S = self._source(rho)
            j = j + 0.5 * S
            feq = equilibrium(rho, j, P)
            psi = np.empty_like(f)
            for i in range(Q):
                psi[i] = self.W[i] * (C[i, 0] * S[0] + C[i, 1] * S[1] + C[i, 2] * S[2]) / self.cs2
            fcol = f - (f - feq) / self.tau + (1 - 1 / (2 * self.tau)) * psi
            self.U += j / rho
            # eq:stream: f_i(x + c_i) = f_col,i(x)
            fnew = np.empty_like(f)
            for i in range(Q):
                fnew[i] = self._neighbour(fcol[i], i, -1)
            if self.walls is not None:
                self._walls(fcol, fnew)
            if self.mask is not None:
                self._links(fcol, fnew)
                # void sites hold the rest state (nothing reads them)
                fnew[:, ~self.mask] = self.rest[:, 0, 0]
                self.U[:, ~self.mask] = 0
            self.f = fnew
            self.n += 1

    def _walls(self, fcol, fnew):
        """Cut links (x, i) at the walls: the population returning to x in
        direction ibar, from the post-collision populations (section 4: eq:bbcon
        and eq:abbcon at q = 1/2, eq:bbnoncon and eq:abbnoncon otherwise).  rho
        and P at x are the step's moments, equal to those of f_col (collision
        conserves both in this closure).  The site behind x along the link,
        x - c_i, is the next site inward (x = 1 or nx - 2); a one-site-wide
        slab has none, and its links lose the terms that need it (q taken as
        1/2), as where two walls cut opposite links in two dimensions."""
        rho, _, P = self._moments(fcol)
        nx = self.shape[2]
        behind = nx >= 2
        for side, (kind, value, q) in enumerate(self.walls):
            value = value * self._factor(self.wprof[side])
            xs = 0 if side == 0 else -1
            normal = np.array([-1.0, 0.0, 0.0]) if side == 0 else np.array([1.0, 0.0, 0.0])
            kappa = (1 - 2 * q) / (1 + 2 * q) if behind else self.dt(0)
            beta = 2 / (1 + 2 * q) if behind else self.dt(1)
            r = rho[:, :, xs]
            Px = P[:, :, :, :, xs]
            for i in range(1, Q):
                # the links this wall cuts: those that leave the material
                # through it (with nx = 1 both walls act on the same sites)
                if C[i, 0] != (-1 if side == 0 else 1):
                    continue
                ib = OPP[i]
                fi = fcol[i, :, :, xs]
                fib = fcol[ib, :, :, xs]
                # f_i at the site behind, x - c_i (wrapped in y and z)
                fi_y = self._neighbour(fcol[i], i, -1)[:, :, xs] if behind else 0
                c = C[i]
                if kind == DIRICHLET:
                    # eq:bbcon / eq:bbnoncon with j* = rho(x) v*
                    jstar = r[None] * value[:, None, None]
                    cj = c[0] * jstar[0] + c[1] * jstar[1] + c[2] * jstar[2]
                    fnew[ib, :, :, xs] = fi + kappa * (fi_y - fib) - beta * 2 * self.W[i] * cj / self.cs2
                else:
                    # eq:abbcon / eq:abbnoncon: rho_bd and the tangential block of the
                    # boundary Cauchy stress at the site, or extrapolated along the
                    # link, (1 + q) X(x) - q X(x - c_i); the normal part from the
                    # traction: sigma* = Pi sigma_b Pi + n t* + t* n - (t*.n) n n
                    sig = self._cauchy(r, Px)
                    rbd = r
                    if behind and self.norder == 1:
                        r_y = self._neighbour(rho, i, -1)[:, :, xs]
                        P_y = np.stack([np.stack([self._neighbour(P[a, b_], i, -1)[:, :, xs]
                                                  for b_ in range(3)]) for a in range(3)])
                        sig = (1 + q) * sig - q * self._cauchy(r_y, P_y)
                        rbd = (1 + q) * r - q * r_y
                    Pi = (np.eye(3) - np.outer(normal, normal)).astype(self.dt)
                    st = np.einsum("ab,bc...,cd->ad...", Pi, sig, Pi)
                    tn = value @ normal
                    for a in range(3):
                        for b_ in range(3):
                            st[a, b_] = st[a, b_] + normal[a] * value[b_] + value[a] * normal[b_] - tn * normal[a] * normal[b_]
                    # eq:bcchainneum with eq:approxdiv at rho_bd
                    Pstar = -st
                    for a in range(3):
                        Pstar[a, a] = Pstar[a, a] + (self.lam - self.mu) * (1.0 - rbd)
                    E = 2 * equilibrium(rbd, np.zeros((3,) + rbd.shape, dtype=self.dt), Pstar)[i]
                    fnew[ib, :, :, xs] = -fi - kappa * (fi_y + fib) + beta * E

    def _links(self, fcol, fnew):
        """The cut links of a general geometry, each with its own q, outward
        normal and group (section 4.2, as `_walls` for planes): the population
        returning to x in direction ibar.  A link whose opposite link at x is
        cut too has no site behind x (kappa = 0, beta = 1, no extrapolation).
        A link through the edge where two faces meet carries both faces'
        groups and normals (the two-dimensional corner reading in three
        dimensions)."""
        rho, _, P = self._moments(fcol)
        L = self.links
        z, y, x, k, q = L["z"], L["y"], L["x"], L["k"], L["q"]
        nz, ny, nx = self.shape
        kb = OPP[k]
        thin = self.cut[kb, z, y, x]
        bz, by, bx = (z - C[k, 2]) % nz, (y - C[k, 1]) % ny, (x - C[k, 0]) % nx
        kappa = np.where(thin, 0, (1 - 2 * q) / (1 + 2 * q))
        beta = np.where(thin, 1, 2 / (1 + 2 * q))
        fk = fcol[k, z, y, x]
        fkb = fcol[kb, z, y, x]
        fky = np.where(thin, 0, fcol[k, bz, by, bx])
        r = rho[z, y, x]
        c = C[k].astype(self.dt)                                   # [m, 3]
        out = np.empty_like(fk)
        gvals = [(v * self._factor(pf), pp * self._factor(pf)) for (v, pp), pf in zip(self.gval, self.gprof)]
        g, g2 = L["g"], L["g2"]
        dirichlet = self.gkind == DIRICHLET
        # where two faces meet on the link (an edge), the Dirichlet face wins
        gd = np.where(dirichlet[g], g, np.where((g2 >= 0) & dirichlet[np.maximum(g2, 0)], g2, -1))
        for gi, (val, pres) in enumerate(gvals):
            sel = gd == gi
            if sel.any():
                # eq:bbcon / eq:bbnoncon with j* = rho(x) v*
                cj = (c[sel] @ val) * r[sel]
                out[sel] = (fk[sel] + kappa[sel] * (fky[sel] - fkb[sel])
                            - beta[sel] * 2 * self.W[k[sel]] * cj / self.cs2)
        sel = gd < 0
        if sel.any():
            # eq:abbcon / eq:abbnoncon.  sigma_b and rho_bd at the site or
            # extrapolated along the link (order 1, not thin)
            sz, sy, sx, sq = z[sel], y[sel], x[sel], q[sel]
            Ps = P[:, :, sz, sy, sx]                              # [3, 3, m]
            rs = rho[sz, sy, sx]
            sig = self._cauchy(rs, Ps)
            rbd = rs
            if self.norder == 1:
                ext = ~thin[sel]
                ry = rho[bz[sel], by[sel], bx[sel]]
                Py = P[:, :, bz[sel], by[sel], bx[sel]]
                sig_y = self._cauchy(ry, Py)
                sig = np.where(ext[None, None], (1 + sq) * sig - sq * sig_y, sig)
                rbd = np.where(ext, (1 + sq) * rs - sq * ry, rs)
            gv = np.array([v for v, _ in gvals], dtype=self.dt).reshape(-1, 3)
            gp = np.array([pp for _, pp in gvals], dtype=self.dt)
            na, ga = L["n"][sel], g[sel]
            ta = gv[ga] - gp[ga][:, None] * na                      # t* = value - pressure n
            st = np.empty_like(sig)
            one = g2[sel] < 0
            if one.any():
                # one face: sigma* = Pi sigma_b Pi + n t* + t* n - (t*.n) n n
                n1, t1, s1 = na[one], ta[one], sig[:, :, one]
                Pi = np.eye(3, dtype=self.dt)[:, :, None] - np.einsum("ma,mb->abm", n1, n1)
                tn = np.einsum("ma,ma->m", t1, n1)
                st[:, :, one] = (np.einsum("abm,bcm,cdm->adm", Pi, s1, Pi) + np.einsum("ma,mb->abm", n1, t1)
                                 + np.einsum("ma,mb->abm", t1, n1) - tn[None, None] * np.einsum("ma,mb->abm", n1, n1))
            if (~one).any():
                # two faces meeting at an edge: in the frame (n_A, n_B, e =
                # n_A x n_B) the tractions fix the rows of n_A and n_B (the
                # shear between them averaged), the edge's own sigma_ee is
                # sigma_b's
                two = ~one
                nA, tA, s2 = na[two], ta[two], sig[:, :, two]
                gb = g2[sel][two]
                nB = L["n2"][sel][two]
                tB = gv[gb] - gp[gb][:, None] * nB
                e = np.cross(nA, nB)
                u = (nA, nB, e)
                dot = lambda a_, b_: np.einsum("ma,ma->m", a_, b_)
                S = {(0, 0): dot(tA, nA), (1, 1): dot(tB, nB), (0, 1): (dot(tA, nB) + dot(tB, nA)) / 2,
                     (0, 2): dot(tA, e), (1, 2): dot(tB, e), (2, 2): np.einsum("ma,abm,mb->m", e, s2, e)}
                acc = np.zeros_like(s2)
                for (i_, j_), v_ in S.items():
                    term = v_[None, None] * np.einsum("ma,mb->abm", u[i_], u[j_])
                    acc = acc + (term if i_ == j_ else term + np.swapaxes(term, 0, 1))
                st[:, :, two] = acc
            Pstar = -st
            for a in range(3):
                Pstar[a, a] = Pstar[a, a] + (self.lam - self.mu) * (1.0 - rbd)
            feq = equilibrium(rbd, np.zeros((3,) + rbd.shape, dtype=self.dt), Pstar)   # [Q, m]
            E = 2 * feq[k[sel], np.arange(len(rbd))]
            out[sel] = -fk[sel] - kappa[sel] * (fky[sel] + fkb[sel]) + beta[sel] * E
        fnew[kb, z, y, x] = out

    # ------------------------------------------------------------ fields
    def init_fields(self, rho=None, vel=None, sigma=None, u=None):
        """f = f_eq(rho, rho v - S/2, P(sigma, rho)), U = u - (j/rho)/2, in
        user units; arrays [nz, ny, nx], vel and u [3, ...], sigma [6, ...]
        (xx, yy, zz, xy, xz, yz)."""
        r = np.ones(self.shape, dtype=self.dt) if rho is None else np.asarray(rho, dtype=self.dt) / self.dt(self.box.rho)
        if not (r > 0).all():
            raise ValueError("density must be positive")
        S = self._source(r)
        j = np.zeros((3,) + self.shape, dtype=self.dt) if vel is None else \
            r * np.asarray(vel, dtype=self.dt) / self.dt(self.s_v)
        sg = np.zeros((3, 3) + self.shape, dtype=self.dt) if sigma is None else \
            sym_to_full(np.asarray(sigma, dtype=self.dt) / self.dt(self.s_sigma))
        P = -sg
        for a in range(3):
            P[a, a] = P[a, a] + (self.lam - self.mu) * (1.0 - r)
        self.f = equilibrium(r, j - 0.5 * S, P)
        u0 = np.zeros((3,) + self.shape, dtype=self.dt) if u is None else np.asarray(u, dtype=self.dt)
        self.U = u0 - 0.5 * j / r
        if self.mask is not None:
            # void sites: the rest state, no displacement (fields there are ignored)
            self.f[:, ~self.mask] = self.rest[:, 0, 0]
            self.U[:, ~self.mask] = 0
        self.n = 0

    def moments(self):
        """(rho [nz,ny,nx], j [3,...], P [6,...], sigma [6,...]) in user units;
        j includes S/2 (eq:moments)."""
        rho, j, P = self._moments(self.f)
        S = self._source(rho)
        j = j + 0.5 * S
        sig = self._cauchy(rho, P)
        sv = self.box.rho * self.s_v
        out = (rho * self.box.rho, j * sv, full_to_sym(P) * self.s_sigma, full_to_sym(sig) * self.s_sigma)
        out = tuple(np.asarray(a, dtype=np.float64) for a in out)
        if self.mask is not None:
            for a in out:
                a[..., ~self.mask] = 0.0            # void sites report zeros
        return out

    def displacement(self):
        """u^n = U^n + (j^n/rho^n)/2: the trapezoid rule for the integral of
        j/rho (U holds u0 - v0/2 plus the left sum), in cells."""
        rho, j, _ = self._moments(self.f)
        j = j + self._source(rho) / 2
        u = np.asarray(self.U + j / rho / 2, dtype=np.float64)
        if self.mask is not None:
            u[:, ~self.mask] = 0.0
        return u

    def populations(self):
        return np.asarray(self.f, dtype=np.float64)

    def set_populations(self, f):
        f = np.asarray(f, dtype=self.dt)
        assert f.shape == (Q,) + self.shape
        self.f = f.copy()
