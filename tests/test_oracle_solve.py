"""Pins of the oracle's whole transmission solve.

* Unit circle: the dense Nystrom solution converges to the Fourier-Bessel
  closed form at third order (Section 6 reports O(h^3) for the Muller-like
  formulations, Fig. helm_error).
* Smooth star: self-convergence at third order.
* The symmetric (row-scaled) and unscaled systems have the same solution:
  W is invertible (Section 3.2).
* Dense LU on tiny inputs: residual at rounding level, and agreement with a
  solve by Cramer's rule on a 2x2 reduced system built by hand.
"""

import numpy as np

import workloads
from oracle import dense, exact, geometry, kernels
from oracle.kernels import Medium


def _solve(x, k0, k1, angle, row_scaled=True):
    g = geometry.discretize(*x)
    med = Medium(k0, k1, 1.0, (k1 / k0) ** 2)
    A = kernels.assemble(g, med, row_scaled)
    uin, qin = dense.plane_wave(g, k0, angle)
    b = dense.rhs(g, med, uin, qin, row_scaled)
    return dense.solve_dense(A, b), A, b


def test_circle_fourier_bessel_third_order():
    errs = []
    for n in (128, 256, 512):
        xs, _, _ = _solve(workloads.circle(n), 10.0, 15.0, 0.0)
        q, u = exact.circle_transmission(n, 10.0, 15.0, 1.0, 2.25, 0.0)
        xe = np.concatenate([q, u])
        errs.append(np.linalg.norm(xs - xe) / np.linalg.norm(xe))
    errs = np.array(errs)
    assert np.all(errs[:-1] / errs[1:] > 7.5), errs
    assert errs[-1] < 5e-5, errs


def test_circle_oblique_incidence():
    n, ang = 256, 0.7
    xs, _, _ = _solve(workloads.circle(n), 4.0, 9.0, ang)
    q, u = exact.circle_transmission(n, 4.0, 9.0, 1.0, (9.0 / 4.0) ** 2, ang)
    xe = np.concatenate([q, u])
    assert np.linalg.norm(xs - xe) / np.linalg.norm(xe) < 2e-4


def test_star_self_convergence():
    sol = {}
    for n in (256, 512, 1024):
        sol[n], _, _ = _solve(workloads.star(n, amp=0.3, arms=5), 10.0, 15.0, 0.4)
    def diff(a, b):
        # nodes of the coarse grid are every other node of the fine grid
        xa, xb = sol[a], sol[b]
        sub = np.concatenate([xb[:b:2], xb[b::2]])
        return np.linalg.norm(xa - sub) / np.linalg.norm(sub)
    d1, d2 = diff(256, 512), diff(512, 1024)
    assert d1 / d2 > 6.5, (d1, d2)
    assert d2 < 5e-4


def test_scaled_and_unscaled_same_solution():
    x = workloads.star(300, amp=0.3, arms=5)
    xs, _, _ = _solve(x, 10.0, 15.0, 1.0, True)
    xb, _, _ = _solve(x, 10.0, 15.0, 1.0, False)
    assert np.linalg.norm(xs - xb) / np.linalg.norm(xs) < 1e-12


def test_dense_lu_tiny():
    rng = np.random.default_rng(5)
    for n in (8, 16, 32, 64):
        xs, A, b = _solve(workloads.star(n, amp=0.2, arms=3), 3.0, 4.0, 0.1)
        assert np.linalg.norm(A @ xs - b) <= 1e-13 * np.linalg.norm(A) * np.linalg.norm(xs)
    # brute force: a 2x2 complex system by Cramer's rule
    M = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    r = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    det = M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
    cr = np.array([(r[0] * M[1, 1] - M[0, 1] * r[1]) / det, (M[0, 0] * r[1] - r[0] * M[1, 0]) / det])
    assert np.allclose(dense.solve_dense(M, r), cr, rtol=1e-13, atol=0)
