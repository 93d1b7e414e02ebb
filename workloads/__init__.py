"""Seeded synthetic inputs shared by the solver's tests, the benchmark and the
oracle: grid faces and surface maps only, no solver arithmetic."""
from . import configs, grids, magnetograms  # noqa: F401
from .configs import C151, C301, SMALL, WORKLOADS, Workload  # noqa: F401
