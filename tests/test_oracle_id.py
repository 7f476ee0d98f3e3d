"""Pins of the oracle's interpolative decomposition (Section 4.1).

* Exact low rank: a product of random complex factors of rank r is recovered
  with k = r and reconstructed to rounding level.
* The column-pivoted QR bound: the ID residual M[:, P[k:]] - M[:, J] T equals
  Q2 R22, so every residual column norm is at most the first rejected pivot,
  <= tol |R_00|.
* Brute force on a tiny matrix: the first skeleton column is the column of
  largest norm.
* Transpose, not conjugate transpose (remark closing Section 4.1): for a
  complex-symmetric matrix a row ID is the transposed column ID, and the
  block A_ij ~= R_i^T S_ij R_j; using R_i^H instead fails.
"""

import numpy as np

from oracle import idec


def _rand(rng, m, n):
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def test_exact_rank_recovered():
    rng = np.random.default_rng(0)
    for (m, n, r) in ((60, 40, 7), (120, 64, 23), (30, 30, 30)):
        M = _rand(rng, m, r) @ _rand(rng, r, n)
        k, perm, T, rd = idec.column_id(M, 1e-12)
        assert k == r
        rec = M[:, perm[:k]] @ T
        if k < n:
            assert np.abs(rec - M[:, perm[k:]]).max() <= 1e-11 * np.abs(M).max()


def test_cpqr_residual_bound():
    rng = np.random.default_rng(1)
    # geometrically decaying singular values
    U, _ = np.linalg.qr(_rand(rng, 150, 80))
    V, _ = np.linalg.qr(_rand(rng, 80, 80))
    M = (U * (0.6 ** np.arange(80))) @ V.conj().T
    for tol in (1e-4, 1e-8, 1e-12):
        k, perm, T, rd = idec.column_id(M, tol)
        res = M[:, perm[k:]] - M[:, perm[:k]] @ T
        colmax = np.sqrt((np.abs(res) ** 2).sum(0)).max() if res.size else 0.0
        assert rd[k - 1] > tol * rd[0]
        # exact arithmetic: colmax = max column norm of R22 <= |R_kk|; forming the
        # residual adds rounding of order eps |M| (1 + |T|)
        slack = 1e-14 * rd[0] * (1.0 + np.abs(T).max())
        assert colmax <= rd[k] + slack, (tol, colmax, rd[k])
        assert rd[k] <= tol * rd[0]


def test_first_pivot_is_largest_column():
    rng = np.random.default_rng(2)
    M = _rand(rng, 6, 4)
    M[:, 2] *= 5.0
    k, perm, T, rd = idec.column_id(M, 1e-14)
    assert perm[0] == 2
    assert np.isclose(rd[0], np.linalg.norm(M[:, 2]))


def test_transpose_not_conjugate():
    rng = np.random.default_rng(3)
    # complex-symmetric matrix with low-rank off-diagonal blocks
    n, r = 40, 5
    B = _rand(rng, n, r) @ _rand(rng, r, n)
    k, perm, T, _ = idec.column_id(B, 1e-12)
    R = idec.interp_matrix(k, perm, T)
    # B ~= B[:, J] R; for C = B^T the row ID is R^T: C ~= R^T C[J, :]
    C = B.T
    J = perm[:k]
    assert np.abs(R.T @ C[J, :] - C).max() < 1e-10 * np.abs(C).max()
    err_conj = np.abs(R.conj().T @ C[J, :] - C).max()
    assert err_conj > 1e-3 * np.abs(C).max()
