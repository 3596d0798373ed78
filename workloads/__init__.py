"""Seeded synthetic inputs shaped like the paper's workloads.

Input generation only: this package holds none of the method's arithmetic and
is shared by the oracle tests, the GPU tests and the benchmark.
"""
from .synth import *  # noqa: F401,F403
