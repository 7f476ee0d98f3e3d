"""PMCHWT and Burton-Miller systems on the GPU against the FP64 oracle.

* Entries (eq. symmetric_pmchwt, eq. naive_pmchwt, eq. bm with columns in
  [q; u] order), including every diagonal with the hypersingular N_k
  correction: blockwise max error / max entry below 2e-12.
* The direct product and the plane-wave right-hand side.
* The row-scaled PMCHWT matrix from the device is exactly symmetric.
* HSS solutions (one-sided ID for the symmetric PMCHWT, two-sided for the
  unscaled PMCHWT and Burton-Miller) against the oracle's dense LU solution
  of the same system within 1e-8 at a ragged size (N = 1600, leaf 128); with
  the paper's fixed-rank schedule on the kite within 3x of the oracle's own
  HSS error at that schedule (fixed ranks do not control the error; the
  oracle's values are stored in tests/golden/kite_fixed_rank_oracle.txt).
"""

import math
import os

import numpy as np
import pytest

import workloads
from oracle import dense
from tests.gpu_common import FORMS, make_solver, oracle_system, rel

pytestmark = pytest.mark.gpu


def _star(n=600, leaf=64):
    return workloads.scaled_config(workloads.config2(), n, leaf=leaf)


@pytest.mark.parametrize("form", [3, 4, 5])
@pytest.mark.parametrize("curve", ["circle", "star"])
def test_entries_vs_oracle(form, curve):
    wl = workloads.scaled_config(workloads.config1(), 600, leaf=64) if curve == "circle" else _star()
    eq, rs = FORMS[form]
    _, _, A, b = oracle_system(wl, rs, eq)
    s = make_solver(wl, form=form)
    n = wl.n
    full = s.eval_entries(np.arange(2 * n), np.arange(2 * n))
    for bi in range(2):
        for bj in range(2):
            blk = slice(bi * n, (bi + 1) * n), slice(bj * n, (bj + 1) * n)
            e = np.abs(full[blk] - A[blk]).max() / np.abs(A[blk]).max()
            # the diagonals alone (corrected values and free terms)
            i = np.arange(n)
            ed = np.abs(full[blk][i, i] - A[blk][i, i]).max() / np.abs(A[blk][i, i]).max()
            print(curve, form, bi, bj, "block err", e, "diagonal err", ed)
            assert e < 2e-12 and ed < 2e-12, (bi, bj, e, ed)
    if form == 3:
        assert np.array_equal(full, full.T)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(2 * n) + 1j * rng.standard_normal(2 * n)
    y = s.matvec_direct(x)
    assert rel(y, A @ x) < 1e-12
    assert rel(s.rhs_plane_wave(wl.angle), b) < 1e-13


@pytest.mark.parametrize("form", [3, 4, 5])
def test_solve_vs_dense(form):
    wl = workloads.scaled_config(workloads.config2(), 1600, leaf=128)
    eq, rs = FORMS[form]
    _, _, A, b = oracle_system(wl, rs, eq)
    s = make_solver(wl, form=form)
    s.compress()
    s.factor()
    x = s.solve(s.rhs_plane_wave(wl.angle))
    e = rel(x, dense.solve_dense(A, b))
    st = s.stats()
    print("form", form, "error vs dense", e, "ranks", st["rank_max"][:8], "entries", st["entries_compress"])
    assert e < 1e-8


def _oracle_fixed_rank_error(form):
    """The oracle's own HSS error on the kite at the same fixed-rank schedule
    (tests/golden/kite_fixed_rank_oracle.txt, written by
    tests/golden/make_kite_fixed_rank.py from oracle.hss only)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kite_fixed_rank_oracle.txt")
    for line in open(path):
        if line.startswith("#"):
            continue
        f, _, _, _, e = line.split()
        if int(f) == form:
            return float(e)
    raise KeyError(form)


@pytest.mark.parametrize("root_max", [0, -1])
@pytest.mark.parametrize("form", [3, 4, 5])
def test_kite_fixed_rank_vs_dense(form, root_max):
    # Fixed ranks do not control the error, and the hypersingular N_k of these
    # systems (condition number O(N)) amplifies the truncation of the paper's
    # schedule: the oracle's own HSS solver at the same schedule lands
    # 2.8e-7 .. 6.2e-7 from the dense solution (against 2.0e-8 for the
    # Muller-like system).  The GPU must stay within 3x of that.  root_max -1
    # compresses every level down to two boxes as the oracle does; the default
    # stops at the first level whose ranks fit the dense top-level system.
    wl = workloads.Workload("kite-n1600", "kite", (), 1600, 2.0, 2.0 * math.sqrt(3.0), 0.0, leaf=128)
    eq, rs = FORMS[form]
    _, _, A, b = oracle_system(wl, rs, eq)
    s = make_solver(wl, form=form, root_max=root_max)
    s.configure(rank_leaf=30, rank_scale=1.15)
    s.compress()
    s.factor()
    x = s.solve(b)
    e = rel(x, dense.solve_dense(A, b))
    ref = _oracle_fixed_rank_error(form)
    print("kite form", form, "root_max", root_max, "error vs dense", e, "oracle HSS at the same schedule", ref)
    assert e <= 3 * ref


def test_symmetric_pmchwt_generates_fewer_entries():
    ent = {}
    for n in (2048, 4096):
        wl = workloads.scaled_config(workloads.config2(), n, leaf=64)
        for form in (3, 4):
            s = make_solver(wl, form=form)
            s.compress()
            s.factor()
            st = s.stats()
            ent[(n, form)] = st["entries_compress"] + st["entries_factor"]
            if n == 2048:
                # both forms reach the same (dense) solution
                eq, rs = FORMS[form]
                _, _, A, b = oracle_system(wl, rs, eq)
                e = rel(s.solve(b), dense.solve_dense(A, b))
                print("N", n, "form", form, "error vs dense", e)
                assert e < 1e-8
    print("entries", ent)
    assert ent[(2048, 3)] < 0.8 * ent[(2048, 4)] and ent[(4096, 3)] < 0.8 * ent[(4096, 4)]
