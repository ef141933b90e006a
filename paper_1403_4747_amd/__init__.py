"""MI355X (gfx950) fast directional BEM for high-frequency 3-D acoustics.

The compute path lives in libfda.so (include/fda.h): host C++ builds the
octree, directional cones and compressed operators; hand-written HIP kernels
run the near field, the upward / M2L / downward passes and GMRES.
"""
from .fda import Batch, FDAError, Mlp, Plan, default_options, inspect, library  # noqa: F401

__version__ = "0.1.0"
