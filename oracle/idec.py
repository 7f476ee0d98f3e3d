"""Interpolative decomposition by column-pivoted QR (paper Section 4.1).

A column ID of M (m x n) picks k skeleton columns J = P[:k] and a k x (n-k)
interpolation matrix T with M[:, P[k:]] ~= M[:, J] T, so that
M ~= M[:, J] [I T] P^T.  It comes from the pivoted QR  M P = Q R  (LAPACK
zgeqp3 through SciPy): T = R11^{-1} R12.  The rank is the number of pivots
with |R_jj| > tol |R_00| (tolerance relative to the first pivot).  A row ID of
M is the column ID of M^T with a plain transpose, never a conjugate
transpose (the remark closing Section 4.1).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def column_id(M, tol: float, rank: int | None = None):
    """Returns (k, perm, T, rdiag).  rank fixes k instead of the tolerance."""
    M = np.asarray(M)
    m, n = M.shape
    if n == 0:
        return 0, np.zeros(0, dtype=np.int64), np.zeros((0, 0), M.dtype), np.zeros(0)
    _, R, P = scipy.linalg.qr(M, mode="economic", pivoting=True)
    rd = np.abs(np.diag(R))
    if rank is None:
        if rd.size == 0 or rd[0] == 0.0:
            k = 0
        else:
            small = np.nonzero(rd <= tol * rd[0])[0]
            k = int(small[0]) if small.size else rd.size
    else:
        k = int(min(rank, rd.size))
    if k == 0:
        T = np.zeros((0, n), dtype=M.dtype)
    elif k == n:
        T = np.zeros((k, 0), dtype=M.dtype)
    else:
        T = scipy.linalg.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
    return k, P.astype(np.int64), T, rd


def interp_matrix(k: int, perm, T):
    """Dense k x n matrix [I T] P^T."""
    n = len(perm)
    Rm = np.zeros((k, n), dtype=np.complex128)
    Rm[np.arange(k), perm[:k]] = 1.0
    Rm[:, perm[k:]] = T
    return Rm
