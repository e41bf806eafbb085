"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package generates meshes, right-hand-side source functions and random
vectors.  It holds none of the multigrid method's arithmetic: no basis
functions, quadrature, assembly, point location or solver steps live here.
Both the HIP library (through its Python binding) and the CPU oracle consume
these inputs; neither side imports the other.
"""

from .meshes import (  # noqa: F401
    Mesh,
    structured_box,
    structured_brick,
    dirichlet_face,
    perturb_interior,
    ball_map,
    scramble,
    config_levels,
    CONFIGS,
    SERVING_POOL,
)
from .sources import (  # noqa: F401
    gaussian_bumps,
    bump_centres_cube,
    bump_centres_ball,
    config_source,
    random_vector,
    random_load,
)
