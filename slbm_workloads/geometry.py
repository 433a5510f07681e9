"""Seeded plate geometries: material mask, cut links, wall fractions and normals.

This module describes *problems*, not the method: it holds no lattice-Boltzmann
arithmetic.  Its output is the input that both the HIP library and the CPU
reference take: a material mask, the list of lattice links that cross a wall
(with the wall fraction q = s_i / l_i, the outward wall normal and the
boundary-condition group), and the boundary-condition groups themselves.

Conventions (paper, section "Local boundary rules for the solid LBM"):

* Sites sit at integer coordinates (ix, iy), 0 <= ix < nx, 0 <= iy < ny;
  site index = iy * nx + ix.
* D2Q9 directions in the order 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1),
  5 (1,1), 6 (-1,1), 7 (-1,-1), 8 (1,-1).  This numbering makes the opposite
  of direction 5 equal to 7, as the paper's example of the bounce-back rule has
  it.
* A link (x, k) is *cut* when the segment from x to x + c_k crosses a wall.
  Its wall fraction is q = s/l in (0, 1], s being the distance from x to the
  crossing along the link and l = |c_k|.  Lattice-conforming plate edges lie
  half-way between sites, so their links have q = 1/2.
* The normal stored with a link is the outward unit normal of the material at
  the crossing point.
* A link whose segment passes exactly through the meeting point of two walls
  (a plate corner, the mouth of an edge crack) carries both walls' groups and
  normals (``group2`` >= 0).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)

DIRICHLET = 1
NEUMANN = 2
PROFILE_STEP = 0
PROFILE_RAMP = 1

LINK_DTYPE = np.dtype([
    ("site", np.int32),
    ("dir", np.int32),
    ("q", np.float64),
    ("group", np.int32),
    ("group2", np.int32),
    ("normal", np.float64, (2,)),
    ("normal2", np.float64, (2,)),
])

_TIE = 1e-9


@dataclasses.dataclass
class BCGroup:
    """One boundary-condition group (paper, Dirichlet and Neumann statements).

    kind   DIRICHLET: ``value`` is the wall velocity du*/dt (user units);
           NEUMANN:   ``value`` is the traction t* = sigma n (user units).
    profile PROFILE_STEP: the value is on from t = 0;
            PROFILE_RAMP: scaled by min(t / ramp_time, 1).
    """
    kind: int
    value: tuple = (0.0, 0.0)
    profile: int = PROFILE_STEP
    ramp_time: float = 0.0


@dataclasses.dataclass
class Plate:
    """A complete problem: grid, material, walls and loads (user units, dx = 1)."""
    nx: int
    ny: int
    lam: float
    mu: float
    rho: float
    tau: float
    mask: np.ndarray            # uint8 [ny, nx], 1 = material
    links: np.ndarray           # LINK_DTYPE [n_links], sorted by (site, dir)
    groups: List[BCGroup]
    force: tuple = (0.0, 0.0)
    periodic_x: bool = False
    periodic_y: bool = False
    name: str = ""
    steps: int = 0              # nominal step count of the workload
    # Neumann-rule extrapolation order: 1 = the paper's (rho_bd and sigma_tt
    # linearly extrapolated along the link), 0 = values at the boundary site
    neumann_order: int = 1

    @property
    def n_sites(self) -> int:
        return self.nx * self.ny

    @property
    def n_material(self) -> int:
        return int(self.mask.sum())


# ---------------------------------------------------------------- walls --

@dataclasses.dataclass
class HLine:
    """Horizontal wall y = y0 over x in [x_lo, x_hi) (half-open)."""
    y0: float
    group: int
    x_lo: float = -np.inf
    x_hi: float = np.inf


@dataclasses.dataclass
class VLine:
    """Vertical wall x = x0 over y in [y_lo, y_hi) (half-open)."""
    x0: float
    group: int
    y_lo: float = -np.inf
    y_hi: float = np.inf


@dataclasses.dataclass
class Circle:
    """Circular hole: sites with |x - c| < R are void."""
    cx: float
    cy: float
    R: float
    group: int


def _line_crossing(px, py, k, wall):
    """Fraction s in (0, 1] where segment p -> p + c_k meets a straight wall,
    the outward normal there, or s = inf when it does not."""
    cx, cy = CX[k], CY[k]
    s = np.full(px.shape, np.inf)
    nrm = np.zeros(px.shape + (2,))
    if isinstance(wall, HLine):
        if cy == 0:
            return s, nrm
        t = (wall.y0 - py) / cy
        xc = px + t * cx
        ok = (t > 0) & (t <= 1) & (xc >= wall.x_lo) & (xc < wall.x_hi)
        s = np.where(ok, t, np.inf)
        nrm[..., 1] = np.where(py < wall.y0, 1.0, -1.0)
    else:
        if cx == 0:
            return s, nrm
        t = (wall.x0 - px) / cx
        yc = py + t * cy
        ok = (t > 0) & (t <= 1) & (yc >= wall.y_lo) & (yc < wall.y_hi)
        s = np.where(ok, t, np.inf)
        nrm[..., 0] = np.where(px < wall.x0, 1.0, -1.0)
    return s, nrm


def _circle_crossing(px, py, k, c: Circle):
    """First entry of segment p -> p + c_k into the hole, when its far end is
    inside the hole (a chord with both ends outside is not a cut link)."""
    cx, cy = float(CX[k]), float(CY[k])
    dx, dy = px - c.cx, py - c.cy
    # the far end's test uses the same expression as the void mask
    ex, ey = (px + cx) - c.cx, (py + cy) - c.cy
    inside_far = ex * ex + ey * ey < c.R ** 2
    a = cx * cx + cy * cy
    b = dx * cx + dy * cy
    cc = dx * dx + dy * dy - c.R * c.R
    disc = np.maximum(b * b - a * cc, 0.0)
    t = (-b - np.sqrt(disc)) / a
    # the far end is inside and the near end outside, so the entry lies on the
    # link; keep rounding at a site that sits on the circle from pushing it off
    t = np.clip(t, 1e-9, 1.0)
    s = np.where(inside_far, t, np.inf)
    wx, wy = px + t * cx, py + t * cy
    nrm = np.stack([(c.cx - wx) / c.R, (c.cy - wy) / c.R], axis=-1)
    return s, nrm


def _wall_group(w, px, py):
    """Group of the wall as seen from each site: a crack line may load its two
    faces differently (``left_group``/``right_group`` or ``below_group``/
    ``above_group``)."""
    if hasattr(w, "left_group"):
        return np.where(px < w.x0, w.left_group, w.right_group).astype(np.int32)
    if hasattr(w, "below_group"):
        return np.where(py < w.y0, w.below_group, w.above_group).astype(np.int32)
    return np.full(px.shape, w.group, dtype=np.int32)


def build_plate(nx, ny, *, lam, mu, rho=1.0, tau, walls: Sequence, groups: Sequence[BCGroup],
                force=(0.0, 0.0), periodic_x=False, periodic_y=False, name="", steps=0,
                neumann_order=1) -> Plate:
    """Material mask and cut-link list for a rectangle of sites with walls.

    Plate edges must be given explicitly as walls (HLine/VLine at -1/2 and
    n - 1/2) on non-periodic axes.
    """
    mask = np.ones((ny, nx), dtype=np.uint8)
    for w in walls:
        if isinstance(w, Circle):
            y0, y1 = max(int(np.floor(w.cy - w.R)), 0), min(int(np.ceil(w.cy + w.R)) + 1, ny)
            x0, x1 = max(int(np.floor(w.cx - w.R)), 0), min(int(np.ceil(w.cx + w.R)) + 1, nx)
            yy, xx = np.mgrid[y0:y1, x0:x1]
            sub = mask[y0:y1, x0:x1]
            sub[(xx - w.cx) * (xx - w.cx) + (yy - w.cy) * (yy - w.cy) < w.R ** 2] = 0
    # only sites within one cell of a wall can own a cut link
    near = np.zeros((ny, nx), dtype=bool)
    for w in walls:
        if isinstance(w, Circle):
            # links are at most sqrt(2) long: only sites within 2 cells of the circle
            y0, y1 = max(int(np.floor(w.cy - w.R)) - 2, 0), min(int(np.ceil(w.cy + w.R)) + 3, ny)
            x0, x1 = max(int(np.floor(w.cx - w.R)) - 2, 0), min(int(np.ceil(w.cx + w.R)) + 3, nx)
            yy, xx = np.mgrid[y0:y1, x0:x1]
            d = np.sqrt((xx - w.cx) ** 2 + (yy - w.cy) ** 2)
            near[y0:y1, x0:x1] |= np.abs(d - w.R) <= 2.0
        elif isinstance(w, HLine):
            y0, y1 = max(int(np.floor(w.y0)) - 1, 0), min(int(np.ceil(w.y0)) + 2, ny)
            x0 = max(int(np.floor(max(w.x_lo, -1e9))) - 2, 0)
            x1 = min(int(np.ceil(min(w.x_hi, 1e9))) + 3, nx)
            near[y0:y1, x0:x1] = True
        else:
            x0, x1 = max(int(np.floor(w.x0)) - 1, 0), min(int(np.ceil(w.x0)) + 2, nx)
            y0 = max(int(np.floor(max(w.y_lo, -1e9))) - 2, 0)
            y1 = min(int(np.ceil(min(w.y_hi, 1e9))) + 3, ny)
            near[y0:y1, x0:x1] = True
    sites = np.flatnonzero((mask.astype(bool) & near).ravel())
    px = (sites % nx).astype(np.float64)
    py = (sites // nx).astype(np.float64)
    recs = []
    for k in range(1, 9):
        best = np.full(sites.shape, np.inf)
        g1 = np.full(sites.shape, -1, dtype=np.int32)
        g2 = np.full(sites.shape, -1, dtype=np.int32)
        n1 = np.zeros(sites.shape + (2,))
        n2 = np.zeros(sites.shape + (2,))
        for w in walls:
            if isinstance(w, Circle):
                s, nrm = _circle_crossing(px, py, k, w)
            else:
                s, nrm = _line_crossing(px, py, k, w)
            gid = _wall_group(w, px, py)
            with np.errstate(invalid="ignore"):
                tie = np.isfinite(s) & (np.abs(s - best) <= _TIE)
            closer = s < best - _TIE
            # a second wall met at the same point: keep it as the corner partner
            g2 = np.where(tie, gid, np.where(closer, -1, g2))
            n2 = np.where(tie[:, None], nrm, np.where(closer[:, None], 0.0, n2))
            g1 = np.where(closer, gid, g1)
            n1 = np.where(closer[:, None], nrm, n1)
            best = np.where(closer, s, best)
        cut = np.isfinite(best)
        if not cut.any():
            continue
        r = np.zeros(int(cut.sum()), dtype=LINK_DTYPE)
        r["site"] = sites[cut]
        r["dir"] = k
        r["q"] = best[cut]
        r["group"] = g1[cut]
        r["group2"] = g2[cut]
        r["normal"] = n1[cut]
        r["normal2"] = n2[cut]
        recs.append(r)
    links = np.concatenate(recs) if recs else np.zeros(0, dtype=LINK_DTYPE)
    links = links[np.lexsort((links["dir"], links["site"]))]
    plate = Plate(nx=nx, ny=ny, lam=lam, mu=mu, rho=rho, tau=tau, mask=mask, links=links,
                  groups=list(groups), force=tuple(force), periodic_x=periodic_x,
                  periodic_y=periodic_y, name=name, steps=steps, neumann_order=neumann_order)
    check_plate(plate)
    return plate


def _shifted(m: np.ndarray, dx: int, dy: int, px: bool, py: bool) -> np.ndarray:
    """out[y, x] = m[y + dy, x + dx], wrapped on periodic axes, False outside."""
    if px:
        m = np.roll(m, -dx, axis=1)
    if py:
        m = np.roll(m, -dy, axis=0)
    out = np.zeros_like(m)
    ny, nx = m.shape
    ddx = 0 if px else dx
    ddy = 0 if py else dy
    ys, yd = (slice(max(ddy, 0), ny + min(ddy, 0)), slice(max(-ddy, 0), ny - max(ddy, 0)))
    xs, xd = (slice(max(ddx, 0), nx + min(ddx, 0)), slice(max(-ddx, 0), nx - max(ddx, 0)))
    out[yd, xd] = m[ys, xs]
    return out


def check_plate(p: Plate) -> None:
    """Every uncut link of a material site must end on a material site."""
    m = p.mask.astype(bool)
    cut = np.zeros((9, p.ny, p.nx), dtype=bool)
    cut[p.links["dir"], p.links["site"] // p.nx, p.links["site"] % p.nx] = True
    for k in range(1, 9):
        bad = m & ~cut[k] & ~_shifted(m, CX[k], CY[k], p.periodic_x, p.periodic_y)
        if bad.any():
            raise ValueError(f"{p.name}: {int(bad.sum())} uncut links in direction {k} leave the material")
    # an isolated site (all eight links cut) is not a solid
    if (m & cut[1:].all(axis=0)).any():
        raise ValueError(f"{p.name}: material site with every link cut")


def edge_walls(nx, ny, left=None, right=None, bottom=None, top=None):
    """Straight plate edges half-way outside the outermost sites (q = 1/2)."""
    w = []
    if left is not None:
        w.append(VLine(-0.5, left))
    if right is not None:
        w.append(VLine(nx - 0.5, right))
    if bottom is not None:
        w.append(HLine(-0.5, bottom))
    if top is not None:
        w.append(HLine(ny - 0.5, top))
    return w


def periodic_box(nx, ny, *, lam, mu, rho=1.0, tau, force=(0.0, 0.0), name="periodic") -> Plate:
    return build_plate(nx, ny, lam=lam, mu=mu, rho=rho, tau=tau, walls=[], groups=[],
                       force=force, periodic_x=True, periodic_y=True, name=name)


def mirror_y(p: Plate) -> Plate:
    """The same problem reflected about the horizontal mid-line."""
    L = p.links.copy()
    x = L["site"] % p.nx
    y = L["site"] // p.nx
    mir = np.array([0, 1, 4, 3, 2, 8, 7, 6, 5])
    L["site"] = (p.ny - 1 - y) * p.nx + x
    L["dir"] = mir[L["dir"]]
    L["normal"][:, 1] *= -1
    L["normal2"][:, 1] *= -1
    L = L[np.lexsort((L["dir"], L["site"]))]
    groups = [dataclasses.replace(g, value=(g.value[0], -g.value[1])) for g in p.groups]
    return dataclasses.replace(p, mask=p.mask[::-1].copy(), links=L, groups=groups,
                               force=(p.force[0], -p.force[1]), name=p.name + "-mirror")


def rotate90(p: Plate) -> Plate:
    """The problem rotated by +90 degrees: (x, y) -> (ny - 1 - y, x)."""
    rot = np.array([0, 2, 3, 4, 1, 6, 7, 8, 5])
    L = p.links.copy()
    x = L["site"] % p.nx
    y = L["site"] // p.nx
    nnx = p.ny
    L["site"] = x * nnx + (p.ny - 1 - y)
    L["dir"] = rot[L["dir"]]
    for f in ("normal", "normal2"):
        v = L[f].copy()
        L[f][:, 0] = -v[:, 1]
        L[f][:, 1] = v[:, 0]
    L = L[np.lexsort((L["dir"], L["site"]))]
    groups = [dataclasses.replace(g, value=(-g.value[1], g.value[0])) for g in p.groups]
    mask = np.empty((p.nx, p.ny), dtype=np.uint8)
    yy, xx = np.mgrid[0:p.ny, 0:p.nx]
    mask[xx, p.ny - 1 - yy] = p.mask
    return dataclasses.replace(p, nx=p.ny, ny=p.nx, mask=mask, links=L, groups=groups,
                               force=(-p.force[1], p.force[0]),
                               periodic_x=p.periodic_y, periodic_y=p.periodic_x,
                               name=p.name + "-rot90")
