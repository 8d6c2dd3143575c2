"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds no arithmetic of the sampling method itself: it only draws
graphs, weights, walk starts and update streams.  Every draw is a pure function
of (seed, stream id, element index) through a SplitMix64 counter hash, computed
with wrapping int64 tensor arithmetic, so the integer-valued draws (Erdos-Renyi
and R-MAT endpoints, uniform weights, permutations) are identical on the CPU
and on a GPU.  Weights that go through floating point (Zipf, lognormal) are
drawn in float64 and may differ in the last unit between devices; every test
therefore hands the same arrays to both sides instead of regenerating them.
"""
from .gen import *  # noqa: F401,F403
