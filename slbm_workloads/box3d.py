"""Three-dimensional inputs: a box of sites, periodic in y and z, either
periodic in x or closed by two walls, planes normal to x that cross the links
leaving the material at a fraction q of their length (q = 1/2: the
lattice-conforming planes x = -1/2 and x = nx - 1/2; in general x = -q and
x = nx - 1 + q).  Each wall carries a Dirichlet wall velocity or a Neumann
traction (user units), applied from the first step.

Description only: no arithmetic of the method.  Seeded initial fields for
tests and benchmarks come from :func:`random_velocity`.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

DIRICHLET = 1
NEUMANN = 2

Vec3 = Tuple[float, float, float]


@dataclass
class Wall3:
    kind: int                      # DIRICHLET (value: wall velocity) or NEUMANN (value: traction)
    value: Vec3 = (0.0, 0.0, 0.0)
    q: float = 0.5                 # fraction of a cut link inside the material, (0, 1]


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

    @property
    def n_sites(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def periodic_x(self) -> bool:
        return self.x_walls is None


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
