"""Seeded synthetic satellite catalogues shared by the tests and the benchmark.

Holds input generation only (element distributions, time grids, CSR lists):
none of the propagation model's arithmetic lives here.
"""
from .catalogue import *  # noqa: F401,F403
