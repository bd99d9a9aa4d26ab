"""Seeded synthetic inputs shared by the oracle and the GPU library.

Holds mesh construction and random fields only; no assembly arithmetic."""

from .configs import (ALL_TYPES, config1, config2, config3, config4, config4_sizes,
                      config5, small_mesh)
from . import meshes

__all__ = ["ALL_TYPES", "config1", "config2", "config3", "config4", "config4_sizes",
           "config5", "small_mesh", "meshes"]
