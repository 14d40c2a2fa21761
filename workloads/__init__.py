"""Seeded synthetic inputs for the CRS spMV path.

This package only *builds inputs*: sparsity patterns, matrix values and
right-hand-side vectors.  It performs no matrix-vector arithmetic, so both the
CPU oracle and the GPU library may consume its arrays without sharing any part
of the method under test.
"""
from .gen import *  # noqa: F401,F403
