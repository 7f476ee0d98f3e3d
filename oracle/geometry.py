"""Nystrom discretisation of a parametrised boundary (paper Section 3.1).

Nodes theta_j = 2 pi j / N.  Quadrature weight w_j = |x'(theta_j)| * 2 pi / N
(trapezoidal rule on the 2 pi-periodic parametrisation).  The unit normal
points into the exterior Omega_0 (Section 2); for a counter-clockwise curve
that is nu = (x2', -x1') / |x'|.  Signed curvature
kappa = (x1' x2'' - x2' x1'') / |x'|^3 (positive on a counter-clockwise
convex curve); it enters only the one-point corrected double-layer diagonal.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Geometry:
    x: np.ndarray      # (N, 2) nodes
    nu: np.ndarray     # (N, 2) unit outward normals
    w: np.ndarray      # (N,) trapezoidal weights |x'| 2pi/N
    kappa: np.ndarray  # (N,) signed curvature
    speed: np.ndarray  # (N,) |x'|

    @property
    def n(self) -> int:
        return self.x.shape[0]


def discretize(x, dx, ddx) -> Geometry:
    x = np.asarray(x, dtype=np.float64)
    dx = np.asarray(dx, dtype=np.float64)
    ddx = np.asarray(ddx, dtype=np.float64)
    n = x.shape[0]
    speed = np.hypot(dx[:, 0], dx[:, 1])
    nu = np.stack([dx[:, 1], -dx[:, 0]], axis=1) / speed[:, None]
    kappa = (dx[:, 0] * ddx[:, 1] - dx[:, 1] * ddx[:, 0]) / speed**3
    w = speed * (2.0 * np.pi / n)
    return Geometry(x=x, nu=nu, w=w, kappa=kappa, speed=speed)
