"""Right-hand sides and dense LU solve of the Muller-like, PMCHWT and
Burton-Miller systems.

Right-hand side (eq. symmetric_muller): [-eps0 W u_in; W q_in] with
q_in = d u_in / d nu.  The paper prints (1/eps0) W q_in in the second row;
repeating the derivation from Green's representation (exterior field plus
incident field for the first rows, their normal derivatives for the second)
gives W d u_in/d nu, and both agree at eps0 = 1, the only value the paper and
the measured workloads use.  The unscaled system (eq. naive_muller) drops W.

Solve: LU with partial pivoting (LAPACK zgetrf / zgetrs through SciPy).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from .geometry import Geometry
from .kernels import Medium


def plane_wave(geom: Geometry, k0: float, angle: float):
    """u_in and q_in = d u_in / d nu at the nodes, for direction (cos a, sin a)."""
    d = np.array([np.cos(angle), np.sin(angle)])
    uin = np.exp(1j * k0 * (geom.x @ d))
    qin = 1j * k0 * (geom.nu @ d) * uin
    return uin, qin


def rhs(geom: Geometry, med: Medium, uin, qin, row_scaled: bool = True, eq: str = "muller"):
    """Right-hand side of the chosen system (row-scaled by W or not).

    muller: [-eps0 u_in; q_in]; pmchwt (eq. naive_pmchwt):
    [-u_in; q_in / eps0]; bm (eq. bm): [-u_in - alpha q_in; 0], alpha = i/k0.
    """
    sc = geom.w if row_scaled else np.ones(geom.n)
    if eq == "muller":
        return np.concatenate([-med.eps0 * sc * uin, sc * qin])
    if eq == "pmchwt":
        return np.concatenate([-sc * uin, sc * qin / med.eps0])
    if eq == "bm":
        al = 1j / med.k0
        return np.concatenate([-sc * (uin + al * qin), np.zeros(geom.n, dtype=np.complex128)])
    raise ValueError(f"unknown system {eq!r}")


def solve_dense(A, b):
    lu, piv = scipy.linalg.lu_factor(A, check_finite=False)
    return scipy.linalg.lu_solve((lu, piv), b, check_finite=False)
