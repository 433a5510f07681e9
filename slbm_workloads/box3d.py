"""Three-dimensional inputs: a box of sites, periodic in y and z, either
periodic in x or closed by two walls, planes normal to x that cross the links
leaving the material at a fraction q of their length (q = 1/2: the
lattice-conforming planes x = -1/2 and x = nx - 1/2; in general x = -q and
x = nx - 1 + q).  Each wall carries a Dirichlet wall velocity or a Neumann
traction (user units), applied from the first step.  Or a box periodic on
every axis with a general geometry: a material mask and cut links, each with
its own q, normal and boundary group (spherical cavities, penny-shaped
cracks).

Description only: no arithmetic of the method.  Seeded initial fields for
tests and benchmarks come from :func:`random_velocity`.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

DIRICHLET = 1
NEUMANN = 2
# time profiles of a wall's or group's value: on from t = 0 (STEP), or scaled
# by min(t / ramp_time, 1) (RAMP)
STEP = 0
RAMP = 1

Vec3 = Tuple[float, float, float]


@dataclass
class Wall3:
    kind: int                      # DIRICHLET (value: wall velocity) or NEUMANN (value: traction)
    value: Vec3 = (0.0, 0.0, 0.0)
    q: float = 0.5                 # fraction of a cut link inside the material, (0, 1]
    profile: int = STEP            # STEP or RAMP (over ramp_time, user units)
    ramp_time: float = 0.0


@dataclass
class Box3:
    nx: int
    ny: int
    nz: int
    lam: float
    mu: float
    tau: float
    rho: float = 1.0
    force: Vec3 = (0.0, 0.0, 0.0)
    # None: periodic in x; else the walls at x = -q and x = nx - 1 + q
    x_walls: Optional[Tuple[Wall3, Wall3]] = None
    name: str = ""
    steps: int = 0
    # Neumann walls: rho_bd and the tangential stress taken at the boundary
    # site (0) or extrapolated along the link from the site behind it (1)
    neumann_order: int = 0
    # general geometry (periodic on every axis, no x_walls): the material
    # mask [nz, ny, nx] (1 = material), one record per cut link (LINK3_DTYPE:
    # a link from a material site whose far end is void) and the groups
    mask: Optional[np.ndarray] = None
    links: Optional[np.ndarray] = None
    groups: Optional[list] = None

    @property
    def n_sites(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_material(self) -> int:
        return self.n_sites if self.mask is None else int(self.mask.sum())

    @property
    def periodic_x(self) -> bool:
        return self.x_walls is None


@dataclass
class BCGroup3:
    """Boundary data of cut links: a wall velocity (DIRICHLET), or a traction
    t* = value - pressure n, n the link's outward normal of the material
    (NEUMANN; a pressure loads a curved cavity uniformly)."""
    kind: int
    value: Vec3 = (0.0, 0.0, 0.0)
    pressure: float = 0.0
    profile: int = STEP            # STEP or RAMP (value and pressure scaled by min(t / ramp_time, 1))
    ramp_time: float = 0.0


@dataclass
class Sphere3:
    """Spherical cavity: sites with |x - c|^2 < R^2 are void."""
    cx: float
    cy: float
    cz: float
    R: float
    group: int


@dataclass
class PennyCrack3:
    """Crack of zero thickness: the disk of radius R around (cx, cy) in the
    plane z = zc (zc not an integer, so that no site lies on it).  Every
    link between two material sites that crosses the disk is cut from both
    sides, each face with its own group: `lower` for the material below
    (outward normal +z), `upper` for the material above (-z)."""
    cx: float
    cy: float
    zc: float
    R: float
    lower: int
    upper: int


# D3Q19 directions in the order of the kernels and the reference
C3 = np.array([[0, 0, 0],
               [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
               [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
               [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)

# one cut link: its site, direction, q, group and outward normal; a link
# through the edge where two faces meet carries the second face's group and
# normal too (group2 = -1: none)
LINK3_DTYPE = np.dtype([("site", "<i4"), ("dir", "<i4"), ("q", "<f8"), ("group", "<i4"),
                        ("normal", "<f8", (3,)), ("group2", "<i4"), ("normal2", "<f8", (3,))], align=True)


def link_records3(rows):
    """LINK3_DTYPE records from (site, dir, q, group, normal) tuples, sorted
    by site and direction, with no second group."""
    rows = sorted(rows, key=lambda r: (r[0], r[1]))
    rec = np.zeros(len(rows), dtype=LINK3_DTYPE)
    for k, (site, d, q, g, n) in enumerate(rows):
        rec[k]["site"], rec[k]["dir"], rec[k]["q"], rec[k]["group"], rec[k]["normal"] = site, d, q, g, n
    rec["group2"] = -1
    return rec


def sphere_box3(nx, ny, nz, spheres, groups, *, lam=0.05, mu=0.05, tau=0.55, rho=1.0,
                force=(0.0, 0.0, 0.0), neumann_order=0, name="", steps=0, cracks=()) -> Box3:
    """A box periodic on every axis with spherical cavities (each inside the
    box, away from its faces) and penny-shaped cracks (PennyCrack3, each
    inside the box and clear of the cavities).  A link from a material site
    x whose far end x + c_i lies in a cavity (the first listed that holds it)
    is cut where it first enters that cavity: q = that fraction of the link,
    normal = the material's outward normal there (towards the centre).  A
    link between material sites that crosses a crack is cut where it
    crosses, with the face's normal and group."""
    zz, yy, xx = np.ogrid[0:nz, 0:ny, 0:nx]
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    label = np.full((nz, ny, nx), -1, dtype=np.int32)
    for k in range(len(spheres) - 1, -1, -1):          # the first listed wins
        sp = spheres[k]
        if not (sp.R < sp.cx < nx - 1 - sp.R and sp.R < sp.cy < ny - 1 - sp.R and sp.R < sp.cz < nz - 1 - sp.R):
            raise ValueError("a cavity must lie inside the box")
        inside = (xx - sp.cx) ** 2 + (yy - sp.cy) ** 2 + (zz - sp.cz) ** 2 < sp.R ** 2
        mask[inside] = 0
        label[inside] = k
    cen = np.array([[sp.cx, sp.cy, sp.cz] for sp in spheres], dtype=float).reshape(-1, 3)
    rad = np.array([sp.R for sp in spheres], dtype=float)
    grp = np.array([sp.group for sp in spheres], dtype=np.int64)
    parts = []
    for i in range(1, len(C3)):
        c = C3[i]
        far = np.roll(label, (-c[2], -c[1], -c[0]), axis=(0, 1, 2))
        z, y, x = np.nonzero((mask == 1) & (far >= 0))
        if len(z) == 0:
            continue
        k = far[z, y, x]
        p = np.stack([x, y, z], axis=1).astype(float)
        p0 = p - cen[k]
        a = float(c @ c)
        b = p0 @ c.astype(float)
        cc = (p0 * p0).sum(1) - rad[k] ** 2
        t = (-b - np.sqrt(np.maximum(b * b - a * cc, 0.0))) / a
        t = np.clip(t, 1e-9, 1.0)
        n = (cen[k] - (p + t[:, None] * c)) / rad[k][:, None]
        n = n / np.linalg.norm(n, axis=1)[:, None]
        rec = np.zeros(len(z), dtype=LINK3_DTYPE)
        rec["site"] = (z * ny + y) * nx + x
        rec["dir"] = i
        rec["q"] = t
        rec["group"] = grp[k]
        rec["normal"] = n
        rec["group2"] = -1
        parts.append(rec)
    for ck in cracks:
        if not (ck.R < ck.cx < nx - 1 - ck.R and ck.R < ck.cy < ny - 1 - ck.R and 0 < ck.zc < nz - 1
                and ck.zc != int(ck.zc)):
            raise ValueError("a crack must lie inside the box, off the lattice planes")
        for i in range(1, len(C3)):
            c = C3[i]
            if c[2] == 0:
                continue
            z0 = int(np.floor(ck.zc)) if c[2] > 0 else int(np.floor(ck.zc)) + 1    # the sites whose link crosses
            y, x = np.mgrid[0:ny, 0:nx]
            t = (ck.zc - z0) / c[2]
            hit = (x + t * c[0] - ck.cx) ** 2 + (y + t * c[1] - ck.cy) ** 2 < ck.R ** 2
            both = (mask[z0] == 1) & (mask[z0 + c[2], (y + c[1]) % ny, (x + c[0]) % nx] == 1)
            yy, xx = np.nonzero(hit & both)
            rec = np.zeros(len(yy), dtype=LINK3_DTYPE)
            rec["site"] = (z0 * ny + yy) * nx + xx
            rec["dir"] = i
            rec["q"] = t
            rec["group"] = ck.lower if c[2] > 0 else ck.upper
            rec["normal"] = (0.0, 0.0, float(c[2]))
            rec["group2"] = -1
            parts.append(rec)
    links = np.concatenate(parts) if parts else np.zeros(0, dtype=LINK3_DTYPE)
    links = links[np.lexsort((links["dir"], links["site"]))]
    return Box3(nx, ny, nz, lam=lam, mu=mu, tau=tau, rho=rho, force=tuple(force), name=name or
                f"spheres{nx}x{ny}x{nz}", steps=steps, neumann_order=neumann_order, mask=mask, links=links,
                groups=list(groups))


def block_box3(nx, ny, nz, lo, hi, face_groups, groups, *, lam=0.05, mu=0.05, tau=0.55, rho=1.0,
               force=(0.0, 0.0, 0.0), neumann_order=0, name="", steps=0) -> Box3:
    """A rectangular block of material, sites lo..hi (inclusive, (x, y, z)),
    in a box periodic on every axis with void around it (at least one site
    on every side).  Its six faces are the lattice-conforming planes half a
    link beyond its outer sites (q = 1/2), each with a group: face_groups
    in the order -x, +x, -y, +y, -z, +z.  A link from an edge site that
    leaves through two faces (a face diagonal at the block's edge) crosses
    both at once, at the edge: it carries both faces' groups and normals."""
    lo, hi = np.asarray(lo), np.asarray(hi)
    if not ((lo >= 1).all() and (hi <= np.array([nx, ny, nz]) - 2).all() and (lo <= hi).all()):
        raise ValueError("the block must leave void on every side")
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = 1
    z, y, x = np.nonzero(mask)
    p = np.stack([x, y, z], axis=1)
    parts = []
    for i in range(1, len(C3)):
        c = C3[i]
        # the faces the link leaves through, per axis
        leaves = np.zeros((len(p), 3), dtype=bool)
        for a in range(3):
            if c[a] > 0:
                leaves[:, a] = p[:, a] == hi[a]
            elif c[a] < 0:
                leaves[:, a] = p[:, a] == lo[a]
        cut = leaves.any(axis=1)
        if not cut.any():
            continue
        L = leaves[cut]
        rec = np.zeros(int(cut.sum()), dtype=LINK3_DTYPE)
        rec["site"] = (z[cut] * ny + y[cut]) * nx + x[cut]
        rec["dir"] = i
        rec["q"] = 0.5
        rec["group2"] = -1
        first = np.full(len(rec), -1)
        for a in range(3):
            if c[a] == 0:
                continue
            side = 1 if c[a] > 0 else 0
            nrm = np.zeros(3)
            nrm[a] = 1.0 if side else -1.0
            g = face_groups[2 * a + side]
            sel1 = L[:, a] & (first < 0)
            sel2 = L[:, a] & (first >= 0)
            rec["group"][sel1] = g
            rec["normal"][sel1] = nrm
            first[sel1] = a
            rec["group2"][sel2] = g
            rec["normal2"][sel2] = nrm
        parts.append(rec)
    links = np.concatenate(parts)
    links = links[np.lexsort((links["dir"], links["site"]))]
    return Box3(nx, ny, nz, lam=lam, mu=mu, tau=tau, rho=rho, force=tuple(force), name=name or
                f"block{nx}x{ny}x{nz}", steps=steps, neumann_order=neumann_order, mask=mask, links=links,
                groups=list(groups))


def cavities_box3(n=256, *, per_axis=4, radius=None, pressure=1e-3, mu=0.05, lam=0.05, tau=0.7, seed=0,
                  steps=1000) -> Box3:
    """n^3 porous solid, periodic on every axis: per_axis^3 spherical cavities
    on a jittered cubic grid (seeded), radius 0.3 of the spacing by default,
    every cavity wall loaded by the pressure pressure*mu (Neumann, order 0)."""
    rng = np.random.default_rng(seed)
    h = n / per_axis
    R = 0.3 * h if radius is None else radius
    sph = []
    for iz in range(per_axis):
        for iy in range(per_axis):
            for ix in range(per_axis):
                j = rng.uniform(-0.1 * h, 0.1 * h, 3)
                sph.append(Sphere3((ix + 0.5) * h + j[0], (iy + 0.5) * h + j[1], (iz + 0.5) * h + j[2], R, 0))
    return sphere_box3(n, n, n, sph, [BCGroup3(NEUMANN, (0.0, 0.0, 0.0), pressure * mu)], lam=lam, mu=mu, tau=tau,
                       neumann_order=0, name=f"cavities{n}", steps=steps)


def periodic_box3(nx, ny, nz, *, lam=0.05, mu=0.05, tau=0.55, rho=1.0, force=(0.0, 0.0, 0.0),
                  name="", steps=0) -> Box3:
    return Box3(nx, ny, nz, lam=lam, mu=mu, tau=tau, rho=rho, force=tuple(force),
                name=name or f"box{nx}x{ny}x{nz}", steps=steps)


def slab3(nx, ny, nz, left: Wall3, right: Wall3, *, lam=0.05, mu=0.05, tau=0.55, rho=1.0,
          force=(0.0, 0.0, 0.0), name="", steps=0, neumann_order=0) -> Box3:
    return Box3(nx, ny, nz, lam=lam, mu=mu, tau=tau, rho=rho, force=tuple(force),
                x_walls=(left, right), name=name or f"slab{nx}x{ny}x{nz}", steps=steps,
                neumann_order=neumann_order)


def cube_pulled(n=256, *, mu=0.05, lam=0.05, load=1e-3, tau=0.55, steps=2000) -> Box3:
    """n^3 slab: face x = -1/2 clamped (zero wall velocity), face x = n - 1/2
    pulled by a step normal traction load*mu, periodic in y and z."""
    return slab3(n, n, n, Wall3(DIRICHLET), Wall3(NEUMANN, (load * mu, 0.0, 0.0)), lam=lam, mu=mu,
                 tau=tau, name=f"cube{n}-clamped-pulled", steps=steps)


def random_velocity(box: Box3, seed: int, amplitude: float, smooth: int = 2) -> np.ndarray:
    """Seeded velocity field [3, nz, ny, nx] (user units): uniform random
    values averaged over `smooth` periodic box filters per axis, so that
    neighbouring sites are correlated (a field the lattice resolves)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, (3, box.nz, box.ny, box.nx))
    for _ in range(smooth):
        for ax in (1, 2, 3):
            v = (np.roll(v, 1, ax) + v + np.roll(v, -1, ax)) / 3.0
    return amplitude * v / max(np.abs(v).max(), 1e-300)
