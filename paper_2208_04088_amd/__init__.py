"""MI355X-native solid lattice-Boltzmann step (Faust et al. 2022) behind a C ABI.

``paper_2208_04088_amd.slbm`` binds ``libslbm.so`` (built from ``csrc/`` by
``paper_2208_04088_amd.build``), including the batched path (``slbm.Batch``);
``paper_2208_04088_amd.slbm3`` binds the three-dimensional step and
``paper_2208_04088_amd.serve`` is the serving loop on top of the batch.
"""
from . import slbm  # noqa: F401

__all__ = ["slbm"]
