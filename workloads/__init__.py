"""Seeded synthetic inputs (matrices, partitions, right-hand sides) for DDPS.

Holds no solver arithmetic; shared by the CPU oracle's tests, the GPU tests
and the benchmark.
"""
from . import pde, configs  # noqa: F401
