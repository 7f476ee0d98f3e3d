"""Batched multi-boundary solves on the GPU: a forest of independent
boundaries of different sizes, curves and wavenumbers compressed, factored
and solved level by level in shared launches.

Parity bar for every boundary of the batch:
* relative error <= 1e-8 against the oracle's dense LU solution of that
  boundary's own system;
* agreement with the same boundary solved alone (one-boundary context) to
  1e-9, since the two runs differ only in how launches are shared.
Also checked: cross-boundary entries are zero, the block-diagonal direct
matvec, trees whose top-level systems sit at different heights, and a batch
of one equal to the single-boundary path."""

import dataclasses

import numpy as np
import pytest

import workloads
from oracle import dense
from tests.gpu_common import make_solver, oracle_system, rel

pytestmark = pytest.mark.gpu


def _batch():
    # uneven sizes (and depths), three curves, three media; ragged leaves
    base = workloads.config2()
    return [
        dataclasses.replace(base, name="b0", curve_params=(("amp", 0.2), ("arms", 3)), n=600, k0=5.0, k1=7.5,
                            angle=0.3, leaf=64),
        workloads.Workload("b1", "circle", (), 1000, 10.0, 15.0, 1.1, leaf=64),
        dataclasses.replace(base, name="b2", n=1536, k0=20.0, k1=30.0, angle=2.0, leaf=64),
    ]


def _solve_batch(wls, form=0, root_max=0):
    from paper_2609_33216_amd import binding
    s = binding.Solver(0)
    s.assemble_batch([wl.boundary() for wl in wls], [(wl.k0, wl.k1, wl.eps0, wl.eps1) for wl in wls],
                     leaf=wls[0].leaf, tol=1e-10, form=form, n_proxy=64, root_max=root_max)
    b = s.rhs_plane_wave_batch([wl.angle for wl in wls])
    s.compress()
    s.factor()
    x = s.solve(b)
    return s, b, x


def _split(v, wls):
    out, o = [], 0
    for wl in wls:
        out.append(v[o:o + 2 * wl.n])
        o += 2 * wl.n
    return out


@pytest.mark.parametrize("root_max", [0, 200])
def test_batch_matches_dense_and_single(root_max):
    wls = _batch()
    s, b, x = _solve_batch(wls, root_max=root_max)
    st = s.stats()
    print("batch ranks", st["rank_max"], "root", st["root_size"], "levels", st["levels"])
    for wl, bt, xt in zip(wls, _split(b, wls), _split(x, wls)):
        g, med, A, bo = oracle_system(wl)
        assert rel(bt, bo) < 1e-14
        xd = dense.solve_dense(A, bo)
        e_dense = rel(xt, xd)
        one = make_solver(wl, root_max=root_max)
        one.compress()
        one.factor()
        x1 = one.solve(bo)
        e_single = rel(xt, x1)
        print(wl.name, "N", wl.n, "vs dense", e_dense, "vs single", e_single)
        assert e_dense < 1e-8
        assert e_single < 1e-9


def test_batch_roots_at_different_heights():
    wls = _batch()
    s, _, _ = _solve_batch(wls, root_max=200)
    # box info per level: boundary, index, lo, hi, is-root
    st = s.stats()
    roots = {}
    for lev in range(1, st["levels"] + 1):
        b = 0
        while True:
            try:
                info = s.box_query(lev, b, 16)
            except Exception:
                break
            if info[4]:
                roots.setdefault(int(info[0]), set()).add(lev)
            b += 1
    assert sorted(roots) == [0, 1, 2]
    assert all(len(v) == 1 for v in roots.values())
    assert len({min(v) for v in roots.values()}) >= 2


def test_batch_entries_block_diagonal_and_matvec():
    wls = _batch()
    from paper_2609_33216_amd import binding
    s = binding.Solver(0)
    s.assemble_batch([wl.boundary() for wl in wls], [(wl.k0, wl.k1, wl.eps0, wl.eps1) for wl in wls], leaf=64)
    n0, n1 = wls[0].n, wls[1].n
    rows = np.array([0, 5, 2 * n0 + 3, 2 * n0 + n1 + 7], dtype=np.int64)
    cols = np.array([1, n0 + 2, 2 * n0 + 4, 2 * n0 + 2 * n1 + 9], dtype=np.int64)
    E = s.eval_entries(rows, cols)
    assert np.all(E[:2, 2:] == 0) and np.all(E[2:, :2] == 0)
    assert np.all(E[2:, 3] == 0)
    g, med, A, _ = oracle_system(wls[1])
    assert abs(E[2, 2] - A[3, 4]) <= 1e-13 * abs(A[3, 4])
    assert abs(E[3, 2] - A[n1 + 7, 4]) <= 1e-13 * abs(A[n1 + 7, 4])
    rng = np.random.default_rng(5)
    xv = rng.standard_normal(2 * s.n) + 1j * rng.standard_normal(2 * s.n)
    y = s.matvec_direct(xv)
    for wl, xt, yt in zip(wls, _split(xv, wls), _split(y, wls)):
        _, _, A, _ = oracle_system(wl)
        assert rel(yt, A @ xt) < 1e-13


def test_batch_of_one_is_the_single_path():
    wl = workloads.scaled_config(workloads.config2(), 1000, leaf=64)
    _, b, x = _solve_batch([wl])
    one = make_solver(wl)
    one.compress()
    one.factor()
    x1 = one.solve(b)
    assert np.array_equal(x, x1)
