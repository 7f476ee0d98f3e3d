"""Write the dense-LU solutions of the five-arm star transmission problem.

The curve r = 1 + 0.3 cos 5t, wavenumbers k0 = 50 / k1 = 75, eps1 = 2.25 and
the seeded plane-wave angle are those of the 32768-node bench workload; only N
changes (8192 and 16384 nodes, i.e. 16384 and 32768 unknowns).  The system is
the row-scaled Muller-like one (eq. symmetric_muller), assembled by the oracle
one block of rows at a time (the entries are those of `kernels.assemble`; only
the temporaries are smaller) and solved by LAPACK LU with partial pivoting.
The unscaled system (eq. naive_muller) has the same solution.

Only `oracle/` and the seeded curve sampler are used.  Run from the repository
root:  python -m tests.golden.make_star5_dense [N ...]
The N = 16384 case needs about 20 GB of memory and some minutes of CPU time.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np
import scipy.linalg

import workloads
from oracle import dense, geometry, kernels
from oracle.kernels import Medium, PointSet

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_path(n: int) -> str:
    return os.path.join(HERE, f"star5_k50-75_n{n}_dense_x.npy")


def solve(n: int, rows_per_block: int = 512) -> np.ndarray:
    wl = workloads.config2_reduced(n)
    x, dx, ddx = wl.boundary()
    g = geometry.discretize(x, dx, ddx)
    med = Medium(wl.k0, wl.k1, wl.eps0, wl.eps1)
    ps = PointSet.boundary(g)
    A = np.empty((2 * n, 2 * n), dtype=np.complex128, order="F")
    t0 = time.time()
    for r0 in range(0, n, rows_per_block):
        r1 = min(n, r0 + rows_per_block)
        A11, A12, A21, A22 = kernels.muller_blocks(ps.take(slice(r0, r1)), ps, med, True)
        A[r0:r1, :n] = A11
        A[r0:r1, n:] = A12
        A[n + r0:n + r1, :n] = A21
        A[n + r0:n + r1, n:] = A22
    t1 = time.time()
    uin, qin = dense.plane_wave(g, wl.k0, wl.angle)
    b = dense.rhs(g, med, uin, qin, True)
    lu, piv = scipy.linalg.lu_factor(A, overwrite_a=True, check_finite=False)
    xs = scipy.linalg.lu_solve((lu, piv), b, check_finite=False)
    t2 = time.time()
    print(f"N={n}: assembly {t1 - t0:.1f} s, LU + solve {t2 - t1:.1f} s", flush=True)
    return xs


def main(argv):
    sizes = [int(a) for a in argv] or [8192, 16384]
    for n in sizes:
        xs = solve(n)
        np.save(golden_path(n), xs, allow_pickle=False)


if __name__ == "__main__":
    main(sys.argv[1:])
