"""MI355X (gfx950) implementation of the hot path of DINO-accelerated geometric MCMC.

The kernels live in ``libdino.so`` (built from ``csrc/`` by ``build.py``); this package
only marshals arguments over its C ABI (``include/dino.h``).
"""
from .api import Context, DinoError, Problem, Server, clear_tuning, tune_set, tuning_table  # noqa: F401

__all__ = ["Context", "Problem", "Server", "DinoError", "tuning_table", "tune_set", "clear_tuning"]
