"""Seeded input generators shared by the GPU path's tests/benchmark and the
CPU oracle.  Holds no simulator arithmetic."""
from . import configs, maps  # noqa: F401
