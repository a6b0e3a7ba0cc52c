"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package builds *inputs only*: grid coordinates of the interior points,
the convex-domain indicator mask, the initial field u0, the named parameter
sets and the source / exact-solution fields of the paper's Example 1.  It holds none of the method's arithmetic (no difference
weights, no matrices, no transforms, no solver), so importing it from both
sides does not couple the oracle to the GPU path.
"""

from .configs import (  # noqa: F401
    Workload,
    CONFIG_NAMES,
    make_config,
    interior_coords,
    domain_mask,
    gaussian_bumps,
    example1_workload,
)
from .example1 import example1_exact, example1_source_field  # noqa: F401
from .three_d import Workload3, make_config3d, ellipsoid_mask, interior_coords3  # noqa: F401
