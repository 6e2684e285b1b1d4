"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

Geometry and random coefficients only; no step of the method lives here."""
from . import lattice, workloads  # noqa: F401
