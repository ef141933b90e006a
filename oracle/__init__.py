"""FP64 CPU oracle for the collocation Burton-Miller BEM (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is the dense definition of the operator that the
fast directional algorithm approximates, plus the closed-form and series
solutions that pin it.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
