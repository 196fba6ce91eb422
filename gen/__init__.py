"""Seeded synthetic inputs (grid operators, frontal matrices, right-hand sides).

Shared by the oracle and the GPU path as inputs only; holds none of the
solver's arithmetic.
"""
from . import grids, fronts  # noqa: F401
