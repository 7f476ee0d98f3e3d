"""GPU parity of the proxy-method IDs (Section 4.1) against the oracle.

For boxes at several levels, the oracle rebuilds the box's proxy matrix M_R
from the planner's proxy circle and near-field lists (its own kernel code),
and the device's skeleton J and interpolation matrix R are checked against:
  * the column-pivoted QR bound: every column of M - M[:, J] R has norm at
    most tol * |R_00| (|R_00| = largest column norm of M); 2x slack for the
    two sides' rounding;
  * the true off-diagonal block row: B = A(rows of every other box's active
    nodes, this box's columns), ||B - B[:, J] R||_2 <= 10 tol ||B||_2;
  * symmetry: L = R^T exactly for the one-sided form (eq. low-rank_R), and
    the block A_ij ~= R_i^T S_ij R_j with the plain transpose (the remark
    closing Section 4.1).
Pivot indices are not compared: ties and rounding may pick other, equally
valid skeletons.
"""

import dataclasses

import numpy as np
import pytest

import workloads
from oracle import geometry, kernels
from oracle.kernels import Medium, PointSet
from tests.gpu_common import make_solver

pytestmark = pytest.mark.gpu


def _setup(wl, root_max=-1):
    s = make_solver(wl, form=0, root_max=root_max)
    s.compress()
    x, dx, ddx = wl.boundary()
    g = geometry.discretize(x, dx, ddx)
    med = Medium(wl.k0, wl.k1, wl.eps0, wl.eps1)
    return s, g, med


def _proxy_matrix(s, g, med, level, box):
    cx, cy, Rp, npx = s.box_query(level, box, 10)
    prox = PointSet.proxy_circle((cx, cy), Rp, int(npx))
    near = [s.box_query(level, box, 11), s.box_query(level, box, 12)]
    cols = [s.box_query(level, box, 0), s.box_query(level, box, 1)]
    halves = []
    for t in range(2):
        src = PointSet.boundary(g, cols[t])
        parts = [kernels.muller_blocks(prox, src, med)[2 * e + t] for e in range(2)]
        for e in range(2):
            if len(near[e]):
                parts.append(kernels.muller_blocks(PointSet.boundary(g, near[e]), src, med)[2 * e + t])
        halves.append(np.vstack(parts))
    return halves, cols


# circle, star: the 1024-thread ID variants (fewer than 128 half matrices per
# launch); star128: 128 leaves, so 256 half matrices per launch at the lowest
# levels, which take the 256-thread variant; bigproxy: 320 proxy points per
# circle, so that proxy matrices have more than 512 rows and are reflected by
# the streamed long-column path.
@pytest.mark.parametrize("wl_name", ["circle", "star", "star128", "bigproxy"])
def test_id_bounds(wl_name):
    if wl_name == "circle":
        wl = workloads.scaled_config(workloads.config1(), 1024, leaf=64)
    elif wl_name == "star":
        wl = workloads.config2_reduced(2048)
    elif wl_name == "star128":
        wl = workloads.scaled_config(workloads.config2(), 8192, leaf=64)
    else:
        wl = dataclasses.replace(workloads.config2_reduced(2048), n_proxy=320)
    tol = wl.tol
    s, g, med = _setup(wl)
    st = s.stats()
    L = st["levels"]
    n = g.n
    if wl_name == "bigproxy":
        cx, cy, Rp, npx = s.box_query(L, 0, 10)
        assert 2 * npx > 512
    levels = {L, max(L - 2, 1), max(st["root_level"], 1)}
    if wl_name == "star128":
        levels = {L, L - 1}  # 128 and 64 boxes: 256 and 128 half matrices
        assert 1 << L == 128
    for level in sorted(levels):
        for box in (0, (1 << level) // 3):
            halves, cols = _proxy_matrix(s, g, med, level, box)
            R, Lm = s.box_interp(level, box)
            kq, ku, krq, kru = s.box_query(level, box, 15)
            assert (kq, ku) == (krq, kru)
            assert np.array_equal(Lm, R.T)  # one-sided: L = R^T, no conjugate
            nq = len(cols[0])
            for h, (M, k, r0, c0, nc) in enumerate(((halves[0], kq, 0, 0, nq),
                                                   (halves[1], ku, kq, nq, len(cols[1])))):
                Rh = R[r0:r0 + k, c0:c0 + nc]
                J = s.box_query(level, box, 4 + h)
                # R^(h) is the identity on the skeleton columns
                assert np.array_equal(Rh[:, J], np.eye(k))
                res = M - M[:, J] @ Rh
                cn = np.sqrt((np.abs(M) ** 2).sum(0))
                rn = np.sqrt((np.abs(res) ** 2).sum(0))
                assert rn.max() <= 2 * tol * cn.max(), (level, box, h, rn.max() / cn.max())
            # true off-diagonal block row of the original system
            rows_eq1 = np.array([i for i in _active_others(s, level, box, 2)])
            rows_eq2 = np.array([i for i in _active_others(s, level, box, 3)])
            rows = np.concatenate([rows_eq1, n + rows_eq2])
            colsg = np.concatenate([cols[0], n + cols[1]])
            B = kernels.entries(g, med, rows, colsg)
            J = np.concatenate([s.box_query(level, box, 4), nq + s.box_query(level, box, 5)])
            err = np.linalg.norm(B - B[:, J] @ R, 2) / np.linalg.norm(B, 2)
            print(wl_name, "level", level, "box", box, "ranks", kq, ku, "block-row error / tol", err / tol)
            assert err <= 10 * tol


def _active_others(s, level, box, what):
    out = []
    for b in range(1 << level):
        if b != box:
            out.extend(s.box_query(level, b, what).tolist())
    return out


def test_symmetric_block_factorisation_transpose():
    """A_ij ~= R_i^T A(J_i, J_j) R_j for two leaf boxes (plain transpose).

    Whether R_i^H would fail depends on how far R is from real; at low
    frequency it is nearly real, so that contrast is pinned on a random
    complex matrix in the oracle's tests instead."""
    wl = workloads.scaled_config(workloads.config2(), 1024, leaf=64)
    s, g, med = _setup(wl)
    L = s.stats()["levels"]
    i, j = 0, 5
    def glob(b):
        c = [s.box_query(L, b, 0), s.box_query(L, b, 1)]
        J = [c[0][s.box_query(L, b, 4)], c[1][s.box_query(L, b, 5)]]
        return np.concatenate([c[0], g.n + c[1]]), np.concatenate([J[0], g.n + J[1]])
    ci, Ji = glob(i)
    cj, Jj = glob(j)
    Ri, _ = s.box_interp(L, i)
    Rj, _ = s.box_interp(L, j)
    Aij = kernels.entries(g, med, ci, cj)
    S = kernels.entries(g, med, Ji, Jj)
    approx = Ri.T @ S @ Rj
    err = np.linalg.norm(Aij - approx) / np.linalg.norm(Aij)
    print("R^T S R error", err)
    assert err < 1e-8
