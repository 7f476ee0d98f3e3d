"""Pins of the reference HSS solver (Section 4) against the dense solve.

* Full rank (tol = 0: every ID keeps every column): the compressed equations
  are exact, so the HSS solution equals the dense one to rounding.
* tol = 1e-10: within 1e-8 of the dense solution (the accuracy target).
* On the symmetric matrix the two-sided ID (row IDs of M_L as well) picks the
  same skeletons as the one-sided one, i.e. L_i = R_i^T (Section 4.1).
* The unscaled baseline compressed two-sided reaches the same solution.
"""

import numpy as np

import workloads
from oracle import dense, geometry, hss, kernels
from oracle.kernels import Medium


def _setup(x, k0, k1, row_scaled=True, angle=0.3):
    g = geometry.discretize(*x)
    med = Medium(k0, k1, 1.0, (k1 / k0) ** 2)
    A = kernels.assemble(g, med, row_scaled)
    uin, qin = dense.plane_wave(g, k0, angle)
    b = dense.rhs(g, med, uin, qin, row_scaled)
    return g, med, b, dense.solve_dense(A, b)


def test_full_rank_is_exact():
    g, med, b, xd = _setup(workloads.star(256, amp=0.3, arms=5), 10.0, 15.0)
    H = hss.ReferenceHSS(g, med, leaf=32, tol=0.0)
    H.compress(); H.factor()
    x = H.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12


def test_tolerance_mode_meets_target():
    g, med, b, xd = _setup(workloads.circle(1024), 10.0, 15.0)
    H = hss.ReferenceHSS(g, med, leaf=64, tol=1e-10)
    H.compress(); H.factor()
    x = H.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8


def test_two_sided_on_symmetric_matrix_picks_same_skeletons():
    g, med, b, xd = _setup(workloads.star(512, amp=0.3, arms=5), 10.0, 15.0)
    H1 = hss.ReferenceHSS(g, med, leaf=64, tol=1e-10)
    H2 = hss.ReferenceHSS(g, med, leaf=64, tol=1e-10, two_sided=True)
    H1.compress(); H2.compress()
    for l1, l2 in zip(H1.boxes[1:], H2.boxes[1:]):
        for b1, b2 in zip(l1, l2):
            for h in range(2):
                assert np.array_equal(b2.rskel[h], b2.cskel[h])
                assert np.array_equal(b1.cskel[h], b2.cskel[h])
    H2.factor()
    x = H2.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8


def test_unscaled_two_sided():
    g, med, b, xd = _setup(workloads.star(512, amp=0.3, arms=5), 10.0, 15.0, row_scaled=False)
    H = hss.ReferenceHSS(g, med, leaf=64, tol=1e-10, two_sided=True, row_scaled=False)
    H.compress(); H.factor()
    x = H.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
