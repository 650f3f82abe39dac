"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package draws initial conditions only.  It holds no force, prediction,
correction or time-step arithmetic, so that the oracle and the HIP path stay
independent of each other while reading identical inputs.
"""
from .plummer import plummer, ensemble_sizes, ensemble  # noqa: F401
from .imf import salpeter_masses, plummer_salpeter  # noqa: F401
