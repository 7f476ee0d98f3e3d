"""Pins of the oracle's PMCHWT and Burton-Miller systems.

1. The hypersingular N_k with its one-point corrected diagonal on the unit
   circle.  The closed-form eigenvalue (i pi k^2/2) J_n'(k) H_n'(k) is missed
   at first order, and the first-order term is known exactly: the punctured
   trapezoidal sum of phi(t)/(4 sin^2(t/2)) keeps -(h/2) phi''(0) / (2 pi),
   i.e. + n^2 / (2 N) on mode n.  With it subtracted the remainder converges
   at third order, which pins every constant of the diagonal (a wrong
   -pi/(6 w^2), kappa^2/(24 pi), logarithm or wavenumber constant would leave
   an O(h) or O(h ln h) remainder).
2. Point-source identities for N_k on the star: for v = G_k(., z),
   z inside:  N_k v - (D*_k + W/2) dv/dnu = 0 (exterior representation),
   z outside: N_k v - (D*_k - W/2) dv/dnu = 0 (interior representation),
   converging at first order (Section 3.1's estimate for N_k).
3. Figure 5's contrast on the unit circle: the Muller-like system converges
   to the Fourier-Bessel solution at O(h^3), PMCHWT (symmetric and
   unscaled) and Burton-Miller at O(h); the two PMCHWT forms give one
   solution; the row-scaled PMCHWT matrix is exactly symmetric.
4. Burton-Miller's sign reading: with the printed +alpha eps0 (D*_k0 + I/2)
   the solution does not approach the transmission solution at all.
5. Star: PMCHWT and Burton-Miller solutions approach the Muller-like one at
   first order.
"""

import numpy as np
import pytest
from scipy import special

import workloads
from oracle import dense, exact, geometry, kernels
from oracle.kernels import Medium

STAR = dict(amp=0.3, arms=5)
MED = Medium(10.0, 15.0, 1.0, 2.25)


@pytest.mark.parametrize("k", [10.0, 15.0])
def test_n_single_circle_exact_first_order_term(k):
    ns = (64, 128, 256, 512)
    for mode in (0, 3, 7):
        raw, rem = [], []
        _, _, eN = exact.circle_eigs(mode, k)
        for n in ns:
            g = geometry.discretize(*workloads.circle(n))
            N = kernels.n_single_operator(g, k)
            v = np.exp(1j * mode * 2 * np.pi * np.arange(n) / n)
            lam = (N @ v / g.w) / v
            assert np.allclose(lam, lam[0], rtol=1e-9, atol=1e-9)  # circulant
            raw.append(abs(lam[0] - eN) / abs(eN))
            rem.append(abs(lam[0] - (eN + mode * mode / (2.0 * n))) / abs(eN))
        raw, rem = np.array(raw), np.array(rem)
        assert np.all(rem[:-1] / rem[1:] > 7.5), (mode, rem)
        assert rem[-1] < 2e-5, (mode, rem)
        if mode:
            # the uncorrected error is first order
            assert np.all(np.abs(raw[1:-1] / raw[2:] - 2.0) < 0.25), (mode, raw)


def test_n_single_point_sources_star():
    res = []
    for n in (128, 256, 512):
        g = geometry.discretize(*workloads.star(n, **STAR))
        row = []
        for k in (10.0, 15.0):
            _, _, Ds = kernels.single_operators(g, k)
            N = kernels.n_single_operator(g, k)
            for z, sign in (((0.1, -0.2), +1.0), ((1.9, 1.2), -1.0)):
                d = g.x - np.asarray(z)
                r = np.hypot(d[:, 0], d[:, 1])
                v = 0.25j * special.hankel1(0, k * r)
                dv = -0.25j * k * special.hankel1(1, k * r) * (d * g.nu).sum(1) / r
                lhs = N @ v - (Ds @ dv + sign * 0.5 * g.w * dv)
                row.append(np.linalg.norm(lhs) / np.linalg.norm(N @ v))
        res.append(row)
    res = np.array(res)
    # first order; a wrong free-term sign would leave an O(1) residual
    assert np.all(res[-1] < 0.04), res
    assert np.all(res[:-1] / res[1:] > 1.9), res


def _circle_solution(n, eq, row_scaled, angle=0.3):
    g = geometry.discretize(*workloads.circle(n))
    A = kernels.assemble(g, MED, row_scaled, eq)
    uin, qin = dense.plane_wave(g, MED.k0, angle)
    b = dense.rhs(g, MED, uin, qin, row_scaled, eq)
    return A, dense.solve_dense(A, b)


def _exact(n, angle=0.3):
    q, u = exact.circle_transmission(n, MED.k0, MED.k1, MED.eps0, MED.eps1, angle)
    return np.concatenate([q, u])


def test_figure5_contrast_circle():
    ns = (128, 256, 512)
    errs = {}
    for eq, rs in (("muller", True), ("pmchwt", True), ("pmchwt", False), ("bm", False), ("bm", True)):
        e = []
        for n in ns:
            A, x = _circle_solution(n, eq, rs)
            xe = _exact(n)
            e.append(np.linalg.norm(x - xe) / np.linalg.norm(xe))
            if eq == "pmchwt" and rs:
                assert np.array_equal(A, A.T)
        errs[(eq, rs)] = np.array(e)
    m = errs[("muller", True)]
    assert np.all(m[:-1] / m[1:] > 7.5) and m[-1] < 5e-5, m
    for key in (("pmchwt", True), ("pmchwt", False), ("bm", False), ("bm", True)):
        e = errs[key]
        assert np.all(e[:-1] / e[1:] > 1.9) and np.all(e[:-1] / e[1:] < 2.6), (key, e)
        assert e[-1] < 0.02, (key, e)
    assert np.allclose(errs[("pmchwt", True)], errs[("pmchwt", False)], rtol=1e-8)
    assert np.allclose(errs[("bm", True)], errs[("bm", False)], rtol=1e-8)


def test_bm_printed_sign_does_not_converge():
    for n in (128, 256):
        g = geometry.discretize(*workloads.circle(n))
        A = kernels.assemble(g, MED, False, "bm")
        _, _, Ds = kernels.single_operators(g, MED.k0, row_scaled=False)
        al = kernels.bm_alpha(MED)
        Ap = A.copy()
        Ap[:n, :n] += 2.0 * al * MED.eps0 * (Ds + 0.5 * np.eye(n))  # flip the sign of the D* term
        uin, qin = dense.plane_wave(g, MED.k0, 0.3)
        b = dense.rhs(g, MED, uin, qin, False, "bm")
        xe = _exact(n)
        good = np.linalg.norm(dense.solve_dense(A, b) - xe) / np.linalg.norm(xe)
        bad = np.linalg.norm(dense.solve_dense(Ap, b) - xe) / np.linalg.norm(xe)
        assert good < 0.05 and bad > 0.5, (n, good, bad)


def test_star_pmchwt_bm_approach_muller():
    diffs = []
    for n in (256, 512):
        g = geometry.discretize(*workloads.star(n, **STAR))
        uin, qin = dense.plane_wave(g, MED.k0, 0.3)
        xs = {}
        for eq, rs in (("muller", True), ("pmchwt", True), ("pmchwt", False), ("bm", False)):
            A = kernels.assemble(g, MED, rs, eq)
            if eq == "pmchwt" and rs:
                assert np.array_equal(A, A.T)
            xs[(eq, rs)] = dense.solve_dense(A, dense.rhs(g, MED, uin, qin, rs, eq))
        xm = xs[("muller", True)]
        assert np.linalg.norm(xs[("pmchwt", True)] - xs[("pmchwt", False)]) < 1e-10 * np.linalg.norm(xm)
        diffs.append([np.linalg.norm(xs[k] - xm) / np.linalg.norm(xm) for k in (("pmchwt", True), ("bm", False))])
    diffs = np.array(diffs)
    assert np.all(diffs[0] / diffs[1] > 1.8), diffs
    assert np.all(diffs[1] < 0.05), diffs


def test_entries_match_assembly_all_systems():
    g = geometry.discretize(*workloads.star(96, **STAR))
    rng = np.random.default_rng(5)
    rows = rng.choice(192, 40, replace=False)
    cols = rng.choice(192, 50, replace=False)
    for eq, rs in (("pmchwt", True), ("pmchwt", False), ("bm", False), ("bm", True)):
        A = kernels.assemble(g, MED, rs, eq)
        assert np.array_equal(kernels.entries(g, MED, rows, cols, rs, eq), A[np.ix_(rows, cols)])
