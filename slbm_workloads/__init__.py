"""Seeded synthetic plates for the solid-LBM hot path (inputs only, no method arithmetic)."""
from .geometry import (BCGroup, Circle, DIRICHLET, HLine, LINK_DTYPE, NEUMANN, PROFILE_RAMP,
                       PROFILE_STEP, Plate, VLine, build_plate, check_plate, edge_walls,
                       mirror_y, periodic_box, rotate90)
from . import configs

__all__ = ["BCGroup", "Circle", "DIRICHLET", "HLine", "LINK_DTYPE", "NEUMANN", "PROFILE_RAMP",
           "PROFILE_STEP", "Plate", "VLine", "build_plate", "check_plate", "edge_walls",
           "mirror_y", "periodic_box", "rotate90", "configs"]
