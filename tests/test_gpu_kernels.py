"""GPU parity of the kernel-level pieces against the oracle, through the C-ABI.

* Bessel functions J0, Y0, J1, Y1 (device code) vs SciPy over z in [1e-4, 2e3]:
  error <= 4e-15 |H_n| (H has no real zeros, so this is a relative bound on
  the Hankel functions that the kernels use).
* Matrix entries of both forms (row-scaled eq. symmetric_muller and unscaled
  eq. naive_muller), including the corrected diagonals and free terms, vs the
  oracle's dense assembly.  Tolerance: 2e-12 relative to the largest entry of
  the sub-block.  The oracle subtracts N_k0 and N_k1 directly, which loses up
  to ~3 digits for adjacent nodes (their 1/(2 pi r^2) parts cancel), so its
  own error bounds the comparison; the device combines those poles
  analytically.
* Symmetry of the device entries: A - A^T = (eps0 + eps1)[[0, -W], [W, 0]].
"""

import numpy as np
import pytest
from scipy import special

import workloads
from tests.gpu_common import make_solver, oracle_system

pytestmark = pytest.mark.gpu


def test_bessel_device():
    from oracle import bessel
    from paper_2609_33216_amd import binding
    s = binding.Solver(0)
    z = np.concatenate([np.geomspace(1e-4, 2e3, 4001), [4.0, 4.0 + 1e-12, 25.0, 25.0 - 1e-12]])
    out = s.eval_bessel(z)
    # the oracle's routine (AMOS hankel1, pinned to mpmath); Cephes j0/y0 lose
    # phase accuracy at large z and are not used as the reference
    h0, h1 = bessel.h0(z), bessel.h1(z)
    e0 = np.abs(out[:, 0] + 1j * out[:, 1] - h0) / np.abs(h0)
    e1 = np.abs(out[:, 2] + 1j * out[:, 3] - h1) / np.abs(h1)
    i = int(np.argmax(np.maximum(e0, e1)))
    print("bessel max err / |H|:", max(e0.max(), e1.max()), "at z =", z[i])
    assert e0.max() < 4e-15 and e1.max() < 4e-15
    # regular part of Y1 at small z: Y1 + 2/(pi z) ~ (z/pi) ln(z/2) for z -> 0
    zs = np.array([1e-6, 1e-4, 1e-2])
    o = s.eval_bessel(zs)
    approx = zs / np.pi * (np.log(zs / 2) + np.euler_gamma - 0.5)
    assert np.all(np.abs(o[:, 4] - approx) <= 1e-3 * np.abs(approx))


@pytest.mark.parametrize("form,row_scaled", [(0, True), (1, False)])
@pytest.mark.parametrize("curve", ["circle", "star"])
def test_entries_vs_oracle(form, row_scaled, curve):
    if curve == "circle":
        wl = workloads.scaled_config(workloads.config1(), 600, leaf=64)
    else:
        wl = workloads.scaled_config(workloads.config2(), 600, leaf=64)
    g, med, A, b = oracle_system(wl, row_scaled)
    s = make_solver(wl, form=form)
    n = wl.n
    rng = np.random.default_rng(7)
    rows = np.concatenate([np.arange(0, 40), n + np.arange(0, 40), rng.integers(0, 2 * n, 80)])
    cols = np.concatenate([np.arange(0, 40), n + np.arange(0, 40), rng.integers(0, 2 * n, 80)])
    got = s.eval_entries(rows, cols)
    ref = A[np.ix_(rows, cols)]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(curve, form, "entries max err / max|A|:", err)
    assert err < 2e-12
    # whole matrix at a smaller size, blockwise relative error
    full = s.eval_entries(np.arange(2 * n), np.arange(2 * n))
    for bi in range(2):
        for bj in range(2):
            blk = slice(bi * n, (bi + 1) * n), slice(bj * n, (bj + 1) * n)
            e = np.abs(full[blk] - A[blk]).max() / np.abs(A[blk]).max()
            assert e < 2e-12, (bi, bj, e)


def test_device_entries_symmetry():
    wl = workloads.scaled_config(workloads.config2(), 400, leaf=64)
    s = make_solver(wl, form=0)
    n = wl.n
    A = s.eval_entries(np.arange(2 * n), np.arange(2 * n))
    x, dx, ddx = wl.boundary()
    w = np.hypot(dx[:, 0], dx[:, 1]) * 2 * np.pi / n
    skew = np.zeros_like(A)
    i = np.arange(n)
    skew[i, n + i] = -(wl.eps0 + wl.eps1) * w
    skew[n + i, i] = (wl.eps0 + wl.eps1) * w
    d = np.abs(A - A.T - skew).max() / np.abs(A).max()
    print("device symmetry defect:", d)
    assert d < 1e-14
