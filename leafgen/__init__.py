"""Seeded synthetic inputs for the leaf FDTD solver: label maps and per-label
(n, k) tables.  Shared by the oracle tests and the GPU path; holds none of
the FDTD method's arithmetic."""
from . import geometry, materials, configs  # noqa: F401
from .configs import Instance  # noqa: F401
