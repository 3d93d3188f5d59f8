"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds problem *data* only: box domains, level ranges, coefficient
fields sampled at lattice nodes, analytic solutions and seeded random vectors.
It contains none of the discretisation's arithmetic (no integration, no
transfer operators, no operator application); both the CPU oracle and the GPU
library receive the same arrays from here.
"""
from .configs import *  # noqa: F401,F403
