"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds no arithmetic of the solver itself: it only produces
boundary parametrisations (point, first and second derivative with respect
to the parameter theta) and the scalar settings of each workload.  Both the
oracle and the GPU path start from these arrays and do all of the method's
arithmetic (normals, curvature, quadrature weights, kernels) on their own.
"""

from .curves import circle, star, kite, sample_curve  # noqa: F401
from .configs import (  # noqa: F401
    Workload,
    config1,
    config2,
    config2_reduced,
    config3_batch,
    config4,
    scaled_config,
)
