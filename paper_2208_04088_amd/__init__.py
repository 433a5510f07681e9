"""MI355X-native solid lattice-Boltzmann step (Faust et al. 2022) behind a C ABI.

``paper_2208_04088_amd.slbm`` binds ``libslbm.so`` (built from ``csrc/`` by
``paper_2208_04088_amd.build``); the batched and served paths live in
``paper_2208_04088_amd.batch`` and ``paper_2208_04088_amd.serve``.
"""
from . import slbm  # noqa: F401

__all__ = ["slbm"]
