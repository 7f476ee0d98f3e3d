"""FP64 CPU oracle for the symmetric Muller-like transmission solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, helpers or constant tables); the two meet only in
the seeded boundary samplers of the ``workloads`` package, which hold none of
the method's arithmetic.

What it computes, and where the paper defines it:
  geometry.py  Nystrom nodes, normals, curvature, trapezoidal weights
               (Section 3.1; weight w_j = |x'_j| 2 pi / N)
  bessel.py    H0^(1), H1^(1) through SciPy's AMOS wrappers
  kernels.py   layer-potential kernels (Section 3.1), one-point corrected
               diagonals, the symmetric Muller-like system (eq. symmetric_muller)
               and the unscaled one (eq. naive_muller), entries at arbitrary
               (proxy) points as used by the proxy method (Section 4.1)
  exact.py     unit-circle closed forms: operator eigenvalues and the
               Fourier-Bessel transmission solution
  dense.py     plane-wave right-hand side and dense LU solve (LAPACK)
  idec.py      interpolative decomposition by column-pivoted QR
  hss.py       reference multilevel HSS solver with one- or two-sided proxy
               IDs (Section 4), for algebra checks only

Readings where the paper is silent or garbled are listed in each function's
docstring.  Every function here is pinned by a ``-m "not gpu"`` test against
closed forms, an independent library (mpmath, SciPy quad) or brute force.
"""
