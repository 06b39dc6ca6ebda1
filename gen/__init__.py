"""Seeded synthetic input generators (no sorting arithmetic)."""
from . import workloads  # noqa: F401
