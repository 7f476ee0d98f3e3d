"""Full-size parity on sampled outputs, degenerate sizes and error paths.

* The five-arm star at its full size (N = 32768, leaf 128, tol 1e-10, the
  default top-level threshold: the configuration bench.py times).  The dense
  system does not fit the host, so the oracle computes sampled rows of A one
  by one: the right-hand side (all rows), sampled entries against the
  device's, and the residual |A x - b| of the GPU solution on sampled rows
  (bar 1e-8 of |b| on those rows).  The device's direct product agrees with
  the oracle's rows, and the symmetric and unscaled two-sided solutions agree.
* The smallest trees: N = 2 leaf (two leaves, the root right above them),
  2 leaf + 1 (ragged), and a small wavenumber, against the dense oracle.
* Error paths, forced from the host: invalid sizes, geometry, materials and
  options return EINVAL; calls out of order return ESTATE; the context stays
  usable after an error.
"""

import numpy as np
import pytest

import workloads
from oracle import dense, geometry, kernels
from oracle.kernels import Medium
from tests.gpu_common import make_solver, oracle_system, rel

pytestmark = pytest.mark.gpu

EINVAL, ESTATE = 1, 4


def _oracle_parts(wl, row_scaled=True):
    x, dx, ddx = wl.boundary()
    g = geometry.discretize(x, dx, ddx)
    med = Medium(wl.k0, wl.k1, wl.eps0, wl.eps1)
    uin, qin = dense.plane_wave(g, wl.k0, wl.angle)
    return g, med, dense.rhs(g, med, uin, qin, row_scaled)


def test_full_size_star5_sampled_rows():
    wl = workloads.config2()
    n = wl.n
    g, med, bo = _oracle_parts(wl)
    s = make_solver(wl)
    b = s.rhs_plane_wave(wl.angle)
    assert rel(b, bo) < 1e-13
    rng = np.random.default_rng(17)
    # sampled entries, diagonal pairs included
    ri = np.concatenate([rng.choice(2 * n, 40, replace=False), [5, n + 5, 2 * n - 1]])
    ci = np.concatenate([rng.choice(2 * n, 40, replace=False), [5, n + 5, 2 * n - 1]])
    got = s.eval_entries(ri, ci)
    ref = kernels.entries(g, med, ri, ci, True)
    assert np.abs(got - ref).max() <= 2e-12 * np.abs(ref).max()
    s.compress()
    s.factor()
    xg = s.solve(b)
    st = s.stats()
    rows = rng.choice(2 * n, 48, replace=False)
    Ar = kernels.entries(g, med, rows, np.arange(2 * n), True)
    r = Ar @ xg - bo[rows]
    e = np.linalg.norm(r) / np.linalg.norm(bo[rows])
    print("N", n, "root", st["root_size"], "sampled residual", e)
    assert e < 1e-8
    # the device's direct product on the same rows
    y = s.matvec_direct(xg)
    assert np.abs(y[rows] - Ar @ xg).max() <= 1e-11 * np.abs(bo).max()
    # the unscaled two-sided baseline solves the same problem
    s2 = make_solver(wl, form=1)
    s2.compress()
    s2.factor()
    x2 = s2.solve(s2.rhs_plane_wave(wl.angle))
    d = rel(x2, xg)
    print("sym vs base", d)
    assert d < 1e-8


@pytest.mark.parametrize("n,leaf,k0", [(128, 64, 10.0), (129, 64, 10.0), (256, 64, 0.5), (96, 48, 3.0)])
@pytest.mark.parametrize("form", [0, 1])
def test_smallest_trees(n, leaf, k0, form):
    wl = workloads.Workload(f"star-n{n}", "star", (("amp", 0.2), ("arms", 3)), n, k0, 1.5 * k0, 0.7, leaf=leaf)
    _, _, A, b = oracle_system(wl, row_scaled=form != 1)
    s = make_solver(wl, form=form)
    s.compress()
    s.factor()
    x = s.solve(b)
    e = rel(x, dense.solve_dense(A, b))
    print(n, leaf, k0, form, "levels", s.stats()["levels"], "err", e)
    assert e < 1e-8


def _status(fn):
    from paper_2609_33216_amd.binding import SymhssError
    with pytest.raises(SymhssError) as ei:
        fn()
    return ei.value.status


def test_error_paths_and_recovery():
    from paper_2609_33216_amd import binding
    wl = workloads.scaled_config(workloads.config1(), 512, leaf=64)
    x, dx, ddx = wl.boundary()
    s = binding.Solver(0)
    # out of order before any assemble
    assert _status(s.compress) == ESTATE
    assert _status(s.factor) == ESTATE
    # invalid sizes, geometry, materials, options
    assert _status(lambda: s.assemble(x[:100], dx[:100], ddx[:100], 10.0, 15.0, leaf=64)) == EINVAL  # N < 2 leaf
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, leaf=4)) == EINVAL
    bad = x.copy()
    bad[7, 0] = np.nan
    assert _status(lambda: s.assemble(bad, dx, ddx, 10.0, 15.0, leaf=64)) == EINVAL
    still = dx.copy()
    still[3] = 0.0
    assert _status(lambda: s.assemble(x, still, ddx, 10.0, 15.0, leaf=64)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, -1.0, 15.0, leaf=64)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, eps0=0.0, leaf=64)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, leaf=64, tol=0.0)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, leaf=64, tol=1.5)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, leaf=64, form=6)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, leaf=64, proxy_ratio=1.0)) == EINVAL
    assert _status(lambda: s.assemble(x, dx, ddx, 10.0, 15.0, leaf=64, n_proxy=4)) == EINVAL
    assert _status(lambda: s._check(s.lib.symhss_configure(s.h, 99, 1))) == EINVAL
    assert _status(lambda: s.configure(mixed=2)) == EINVAL
    assert _status(lambda: s.configure(rank_scale=0.5)) == EINVAL
    # a valid assemble afterwards; stages still enforced
    s.assemble(x, dx, ddx, wl.k0, wl.k1, leaf=64)
    b = s.rhs_plane_wave(0.3)
    assert _status(lambda: s.solve(b)) == ESTATE
    assert _status(s.factor) == ESTATE
    s.compress()
    assert _status(lambda: s.solve(b)) == ESTATE
    s.factor()
    x1 = s.solve(b)
    # re-assembling invalidates the later stages
    s.assemble(x, dx, ddx, wl.k0, wl.k1, leaf=64)
    assert _status(lambda: s.solve(b)) == ESTATE
    s.compress()
    s.factor()
    assert np.array_equal(s.solve(b), x1)
