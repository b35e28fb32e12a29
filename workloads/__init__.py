"""Seeded synthetic inputs for the Nystrom-Schur solver and its oracle.

This package builds matrices, partitions, sketches and right-hand sides.  It
holds none of the method's arithmetic: it only produces the inputs that both
the GPU library and the CPU oracle consume, so that the two sides see exactly
the same problem.
"""

from .grids import (  # noqa: F401
    GridProblem,
    box_ids_1d,
    diffusion_fd,
    aniso_problem,
    anisotropic_q1,
    lognormal_field,
    partition_boxes,
    level2_labels,
    sketch,
    rhs,
    make_problem,
    config_c0,
    config_c1,
    config_c2,
    config_c3_problem,
    config_c4,
    config_c5,
    CONFIGS,
    random_dbbd,
    laplacian,
)
