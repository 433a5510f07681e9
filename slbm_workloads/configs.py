"""Synthetic workloads of the solid-LBM hot path, built from seeds.

Every workload is a :class:`~slbm_workloads.geometry.Plate` in user units
with dx = 1 cell and density rho = 1.  Loads are expressed as fractions of
the shear modulus mu.  Nothing here depends on the lattice-Boltzmann method;
the module only states problems.

Relaxation time rule: tau_bar = 0.55 (the value the paper adopts) when
lambda/mu <= 1.5, and 0.6 above, where 0.55 is linearly unstable in the bulk.

Neumann extrapolation: the long synthetic workloads (thousands of steps) take
``neumann_order=0`` -- boundary density and tangential stress taken at the
boundary site -- because the paper's linear extrapolation along the link
drives a growing surface mode on traction-free walls (about 0.8 % per step at
lambda = mu, tau_bar = 0.55) that the paper's short runs do not reach.  The
paper-scale reruns keep the paper's rule (``neumann_order=1``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from .geometry import (BCGroup, Circle, DIRICHLET, HLine, NEUMANN, PROFILE_RAMP,
                       PROFILE_STEP, Plate, VLine, build_plate, edge_walls)


def tau_for(lam_over_mu: float) -> float:
    return 0.55 if lam_over_mu <= 1.5 else 0.6


def square_clamped_pulled(n: int = 128, *, mu: float = 0.05, lam: float = 0.05,
                          load: float = 1e-3, steps: int = 2000, tau: float = 0.55,
                          neumann_order: int = 0) -> Plate:
    """n x n plate: left edge u = 0 (lattice-conforming Dirichlet), right edge a
    step traction sigma_xx = load*mu, top and bottom traction-free."""
    groups = [BCGroup(DIRICHLET, (0.0, 0.0)),          # 0 left, clamped
              BCGroup(NEUMANN, (load * mu, 0.0)),      # 1 right, pulled
              BCGroup(NEUMANN, (0.0, 0.0))]            # 2 top/bottom, free
    walls = edge_walls(n, n, left=0, right=1, bottom=2, top=2)
    return build_plate(n, n, lam=lam, mu=mu, tau=tau, walls=walls, groups=groups,
                       name=f"square{n}-clamped-pulled", steps=steps,
                       neumann_order=neumann_order)


def edge_crack_plate(nx: int = 1024, ny: int = 512, crack: int = 256, *, mu: float = 0.05,
                     lam: float = 0.05, load: float = 1e-3, steps: int = 10000,
                     tau: float = 0.55, neumann_order: int = 0) -> Plate:
    """nx x ny plate with a traction-free crack of ``crack`` cells entering from
    the left edge at mid-height (the line y = ny/2 - 1/2, between two rows).
    Top and bottom carry a step tensile traction sigma_yy = load*mu.  The crack
    occupies x in [-1/2, crack - 1/2): the diagonal link through the tip point
    is not cut."""
    yc = ny / 2 - 0.5
    groups = [BCGroup(NEUMANN, (0.0, 0.0)),            # 0 free edges and crack faces
              BCGroup(NEUMANN, (0.0, load * mu)),      # 1 top, pulled up
              BCGroup(NEUMANN, (0.0, -load * mu))]     # 2 bottom, pulled down
    walls = edge_walls(nx, ny, left=0, right=0, bottom=2, top=1)
    walls.append(HLine(yc, 0, x_lo=-0.5, x_hi=crack - 0.5))
    plate = build_plate(nx, ny, lam=lam, mu=mu, tau=tau, walls=walls, groups=groups,
                        name=f"crack{nx}x{ny}-a{crack}", steps=steps,
                        neumann_order=neumann_order)
    plate.crack_tip_x = crack - 0.5
    return plate


def hole_plate(n: int = 2048, R: float = 256.0, *, mu: float = 0.05, lam: float = 0.1,
               load: float = 1e-3, steps: int = 20000, tau=None,
               neumann_order: int = 0) -> Plate:
    """n x n plate with a centred circular hole of radius R (curved wall, q from
    the exact circle).  Left and right edges carry a step tension load*mu;
    top, bottom and the hole are traction-free."""
    c = (n - 1) / 2.0
    groups = [BCGroup(NEUMANN, (0.0, 0.0)),
              BCGroup(NEUMANN, (load * mu, 0.0)),      # right, pulled +x
              BCGroup(NEUMANN, (-load * mu, 0.0))]     # left, pulled -x
    walls = edge_walls(n, n, left=2, right=1, bottom=0, top=0)
    walls.append(Circle(c, c, R, 0))
    return build_plate(n, n, lam=lam, mu=mu, tau=tau if tau is not None else tau_for(lam / mu),
                       walls=walls, groups=groups, name=f"hole{n}-R{R:g}", steps=steps,
                       neumann_order=neumann_order)


def moving_hole_plate(n: int = 2048, *, mu: float = 0.05, lam: float = 0.04, tau: float = 0.55,
                      wall_speed=(1e-4, -2e-4), ramp_steps: int = 2000, force=(1e-6, -2e-6),
                      steps: int = 20000) -> Plate:
    """Periodic n x n plate (no edges) with two holes, both curved Dirichlet
    walls: one held fixed (u* = 0, radius 0.18 n, centred at (0.45 n,
    0.55 n)) against which a uniform body force presses the material, and a
    smaller one (radius 0.1 n, at (0.8 n, 0.25 n)) whose wall moves with a
    velocity ramped from zero over ramp_steps steps and then held, so that
    its links carry j* = rho du*/dt != 0 (the paper's curved Dirichlet rule,
    section 4.2).  No wall is traction-free, so the plate stays stable."""
    dt = math.sqrt(1.0 / (3.0 * mu))
    groups = [BCGroup(DIRICHLET, (0.0, 0.0)),
              BCGroup(DIRICHLET, tuple(wall_speed), PROFILE_RAMP, ramp_steps * dt)]
    walls = [Circle(n * 0.45, n * 0.55, n * 0.18, 0), Circle(n * 0.8, n * 0.25, n * 0.1, 1)]
    return build_plate(n, n, lam=lam, mu=mu, tau=tau, walls=walls, groups=groups, force=tuple(force),
                       periodic_x=True, periodic_y=True, name=f"movinghole{n}", steps=steps,
                       neumann_order=0)


# ----------------------------------------------------------- paper scale --

def paper_hole_plate(c2_ratio: float = 3.0, *, n: int = 80, mu: float = 1.0,
                     rho: float = 1.0) -> Plate:
    """The paper's plate with a circular hole (r = 0.133 l) at dx = l/80: top
    and bottom loaded in their normal directions by a traction ramped from 0 at
    t = 0 to 5 mu u_ref/l at t = l/c_s (u_ref = 1e-3 l), then held, until
    t = 2 l/c_s.  c2_ratio = c_d^2/c_s^2 = (lambda + 2 mu)/mu."""
    lam = (c2_ratio - 2.0) * mu
    l = float(n)
    cs = math.sqrt(mu / rho)
    t_ramp = l / cs
    t_load = 5.0 * mu * 1e-3
    c = (n - 1) / 2.0
    groups = [BCGroup(NEUMANN, (0.0, 0.0)),
              BCGroup(NEUMANN, (0.0, t_load), PROFILE_RAMP, t_ramp),
              BCGroup(NEUMANN, (0.0, -t_load), PROFILE_RAMP, t_ramp)]
    walls = edge_walls(n, n, left=0, right=0, bottom=2, top=1)
    walls.append(Circle(c, c, 0.133 * l, 0))
    dt = math.sqrt(rho / (3.0 * mu))
    return build_plate(n, n, lam=lam, mu=mu, rho=rho, tau=0.55, walls=walls, groups=groups,
                       name=f"paper-hole{n}-c2r{c2_ratio:g}", steps=int(round(2.0 * l / cs / dt)))


def paper_center_crack(*, n: int = 400, crack: int = 100, mu: float = 1.3, rho: float = 1.0,
                       cs2_over_cd2: float = 0.3611, t_face: float = 0.009615) -> Plate:
    """The paper's stationary crack: a square of side 4 l_c with a centred crack
    of length l_c along y, dx = l_c/100; both crack faces suddenly loaded by a
    traction t* = t_face*mu pushing along their inward normals (mode I opening)."""
    lam = (1.0 / cs2_over_cd2 - 2.0) * mu
    x_c = (n - 1) / 2.0           # the crack line lies between two columns
    y_lo = (n - crack) / 2.0 - 0.5
    t = t_face * mu
    # traction on a face with outward normal n is t = -t* n (pressure opening the crack)
    groups = [BCGroup(NEUMANN, (0.0, 0.0)),
              BCGroup(NEUMANN, (-t, 0.0)),    # left face: outward normal +x, pushed to -x
              BCGroup(NEUMANN, (t, 0.0))]     # right face: outward normal -x, pushed to +x
    walls = edge_walls(n, n, left=0, right=0, bottom=0, top=0)
    # one VLine per face so that each side gets its own load: sites left of
    # the line see outward normal +x
    walls.append(_FaceVLine(x_c, y_lo, y_lo + crack, left_group=1, right_group=2))
    cd = math.sqrt((lam + 2 * mu) / rho)
    dt = math.sqrt(rho / (3.0 * mu))
    return build_plate(n, n, lam=lam, mu=mu, rho=rho, tau=0.55, walls=walls, groups=groups,
                       name=f"paper-crack{n}", steps=int(round(2.0 * crack / cd / dt)))


@dataclasses.dataclass
class _FaceVLine(VLine):
    """A vertical crack line whose two faces belong to different groups."""
    left_group: int = 0
    right_group: int = 0

    def __init__(self, x0, y_lo, y_hi, left_group, right_group):
        super().__init__(x0, left_group, y_lo, y_hi)
        self.left_group = left_group
        self.right_group = right_group


# ------------------------------------------------------- random plates --

def _random_plate(rng: np.random.Generator, *, area_lo: float, area_hi: float,
                  load: float, steps: int, name: str) -> Plate:
    A = math.exp(rng.uniform(math.log(area_lo), math.log(area_hi)))
    a = rng.uniform(1.0, 2.0)
    nx = max(int(round(math.sqrt(A * a))), 16)
    ny = max(int(round(A / nx)), 16)
    mu = rng.uniform(0.02, 0.08)
    lm = rng.uniform(0.5, 2.0)
    lam = lm * mu
    crack = None
    if rng.uniform() < 0.5:
        L = int(round(rng.uniform(0.1, 0.4) * nx))
        yc = math.floor(rng.uniform(0.25, 0.75) * ny) + 0.5
        crack = (L, yc)
    holes = []
    n_holes = int(rng.integers(0, 4))
    tries = 0
    while len(holes) < n_holes and tries < 200:
        tries += 1
        R = rng.uniform(0.05, 0.2) * nx
        if nx - 1 - R - 3 <= R + 3 or ny - 1 - R - 3 <= R + 3:
            continue                   # no room for this radius (small plates)
        cx = rng.uniform(R + 3, nx - 1 - R - 3)
        cy = rng.uniform(R + 3, ny - 1 - R - 3)
        if cx - R < 3 or cy - R < 3 or cy + R > ny - 4 or cx + R > nx - 4:
            continue
        ok = all(math.hypot(cx - h[0], cy - h[1]) > R + h[2] + 3 for h in holes)
        if ok and crack is not None:
            L, yc = crack
            dx = max(cx - (L - 0.5), 0.0)
            ok = math.hypot(dx, cy - yc) > R + 3
        if ok:
            holes.append((cx, cy, R))
    groups = [BCGroup(NEUMANN, (0.0, 0.0)),
              BCGroup(NEUMANN, (load * mu, 0.0)),
              BCGroup(NEUMANN, (-load * mu, 0.0))]
    walls = edge_walls(nx, ny, left=2, right=1, bottom=0, top=0)
    if crack is not None:
        walls.append(HLine(crack[1], 0, x_lo=-0.5, x_hi=crack[0] - 0.5))
    for (cx, cy, R) in holes:
        walls.append(Circle(cx, cy, R, 0))
    return build_plate(nx, ny, lam=lam, mu=mu, tau=tau_for(lm), walls=walls, groups=groups,
                       name=name, steps=steps, neumann_order=0)


def batch_plates(seed: int = 0, count: int = 64, steps: int = 5000) -> List[Plate]:
    """Independent plates of uneven size and geometry: area log-uniform in
    [128^2, 1024^2], aspect in [1, 2], 0-3 holes of radius 5-20 % of the
    width, an edge crack of 10-40 % of the width with probability 1/2,
    mu ~ U[0.02, 0.08], lambda/mu ~ U[0.5, 2], step tension 1e-3 mu on the
    left and right edges."""
    rng = np.random.default_rng(seed)
    return [_random_plate(rng, area_lo=128 ** 2, area_hi=1024 ** 2, load=1e-3, steps=steps,
                          name=f"batch{seed}-{i}") for i in range(count)]


@dataclasses.dataclass
class Request:
    arrival: float      # seconds after the trace starts
    plate: Plate
    steps: int


def served_trace(seed: int = 1, count: int = 256, rate: float = 50.0,
                 area_lo: float = 256 ** 2, area_hi: float = 4096 ** 2) -> List[Request]:
    """Poisson arrivals of plate solves: size log-uniform in [256^2, 4096^2],
    geometry as for :func:`batch_plates`, traction U[1e-4, 1e-3]*mu, step
    count log-uniform in [1e3, 2e4]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        load = rng.uniform(1e-4, 1e-3)
        steps = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e4)))))
        p = _random_plate(rng, area_lo=area_lo, area_hi=area_hi, load=load, steps=steps,
                          name=f"req{seed}-{i}")
        out.append(Request(t, p, steps))
    return out
