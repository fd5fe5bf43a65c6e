"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds geometry and parameter generation only (no time-step arithmetic);
see `configs` for the workload recipes.
"""
from . import configs, geometry  # noqa: F401
