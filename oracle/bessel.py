"""Hankel functions of the first kind, orders 0 and 1, through SciPy (AMOS).

G_k(x, y) = (i/4) H0^(1)(k |x - y|) is the 2-D fundamental solution
(Section 3.1).  The oracle calls the library routine and adds nothing of its
own; the tests pin it against mpmath at high precision and the Wronskian.
"""

from __future__ import annotations

import numpy as np
from scipy import special


def h0(z):
    return special.hankel1(0, np.asarray(z, dtype=np.float64))


def h1(z):
    return special.hankel1(1, np.asarray(z, dtype=np.float64))


def jy01(z):
    """(J0, Y0, J1, Y1) at real z > 0."""
    z = np.asarray(z, dtype=np.float64)
    return special.j0(z), special.y0(z), special.j1(z), special.y1(z)
