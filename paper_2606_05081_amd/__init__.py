"""MI355X-native BVSS breadth-first search (BLEST hot path) for gfx950.

Submodules:
  blest   -- Python binding of the C ABI (include/blest.h); imports torch.
  inputs  -- seeded synthetic graph generators (no torch).
  switch  -- learned engine-switch pipeline (dataset, training, evaluation).
  autotune -- launch/structure parameter search with a JSON cache.
"""
import importlib

__all__ = ["blest", "inputs", "switch", "autotune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
