"""Reference multilevel HSS direct solver (paper Section 4), plain NumPy.

For algebra checks only: it approximates the dense solution, it never stands
in for it.  The steps follow Section 4 in order.

Tree.  A perfect binary tree over contiguous index ranges of the nodes
(the partition into p subsets of Section 4.1), halving each range; level L
holds the leaves, level 0 the root.

Proxy method (Section 4.1, Table tab:observation).  Each box b at level l has
a centre c_b (midpoint of the bounding box of its nodes) and radius r_b (the
largest node distance from c_b).  Gamma'_b is the union of a proxy circle of
radius R_p = ratio * r_b with n_p points and the near field: the active
points of the other boxes of level l closer than R_p to c_b.  M_R has the
observation points Gamma'_b (two rows per point, one per equation) and the
box's active points as sources; M_L the reverse.

One-sided (symmetric) compression, eq. low-rank_R: column IDs of the q-half
and the u-half of M_R give R_b = diag(R_b^(1), R_b^(2)) and L_b = R_b^T.
Two-sided compression, eq. low-rank: additionally row IDs of the two halves
of M_L give L_b.  A two-sided box uses the larger of its row and column rank
in each half so that the compressed blocks stay square.

Compressed equations (Section 4.2): with D_b the diagonal block,
X_b = D_b^{-1} L_b, A~_b = (R_b X_b)^{-1}; the right-hand side becomes
A~_b R_b D_b^{-1} f_b and the solution is recovered from
x_b = D_b^{-1} f_b - X_b (f~_b - A~_b y_b).

Multilevel reading (the paper defers the details to an earlier paper): the
active points of a parent are the union of its children's skeletons, kept
separately for the two halves; the parent's diagonal block is
[[A~_c1, S_c1c2], [S_c2c1, A~_c2]] with S the original matrix entries between
skeletons; the levels L..1 are compressed and the level-0 system is solved
densely.  Proxy count: n_p = max(n_min, 2 ceil(k1 R_p) + 24) rounded up to a
multiple of 16.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg

from .geometry import Geometry
from .kernels import Medium, PointSet, system_blocks
from .idec import column_id, interp_matrix


def tree_ranges(n: int, leaf: int):
    """levels[l] = list of (lo, hi) index ranges, l = 0..L."""
    L = max(1, math.ceil(math.log2(n / leaf))) if n > leaf else 1
    levels = [[(0, n)]]
    for _ in range(L):
        nxt = []
        for lo, hi in levels[-1]:
            mid = (lo + hi) // 2
            nxt.append((lo, mid))
            nxt.append((mid, hi))
        levels.append(nxt)
    return levels


def proxy_count(k1: float, radius: float, n_min: int) -> int:
    n = max(n_min, 2 * math.ceil(k1 * radius) + 24)
    return 16 * math.ceil(n / 16)


@dataclasses.dataclass
class Box:
    lo: int
    hi: int
    center: np.ndarray
    radius: float
    # active point lists (node indices) for the two halves, rows and columns
    rows: list = None   # [eq1 rows, eq2 rows]
    cols: list = None   # [q cols, u cols]
    rskel: list = None
    cskel: list = None
    R: np.ndarray = None   # (kc, ncols)  column interpolation  [I T]P^T per half
    L: np.ndarray = None   # (nrows, kr)  row interpolation
    D: np.ndarray = None
    X: np.ndarray = None
    At: np.ndarray = None  # A~
    lu: tuple = None
    ranks: tuple = None


class ReferenceHSS:
    """eq selects the system ("muller", "pmchwt" or "bm", as in kernels.system_blocks);
    only the row-scaled Muller-like and PMCHWT systems are symmetric.  rank fixes
    every ID's rank; schedule = (k_L, a) gives a box at level l the rank
    round(k_L a^(L - l)) (Section 4.3) instead of the tolerance rule."""

    def __init__(self, geom: Geometry, med: Medium, leaf: int, tol: float,
                 two_sided: bool = False, row_scaled: bool = True,
                 n_proxy_min: int = 64, proxy_ratio: float = 1.5, rank: int | None = None,
                 eq: str = "muller", schedule: tuple | None = None):
        if not two_sided and (not row_scaled or eq == "bm"):
            raise ValueError("a non-symmetric system needs two_sided=True")
        self.g, self.med, self.eq = geom, med, eq
        self.tol, self.two_sided, self.row_scaled = tol, two_sided, row_scaled
        self.n_proxy_min, self.ratio, self.fixed_rank = n_proxy_min, proxy_ratio, rank
        self.schedule = schedule
        self.ranges = tree_ranges(geom.n, leaf)
        self.L = len(self.ranges) - 1
        self.boxes = []
        for lev in self.ranges:
            row = []
            for lo, hi in lev:
                pts = geom.x[lo:hi]
                c = 0.5 * (pts.min(axis=0) + pts.max(axis=0))
                r = float(np.sqrt(((pts - c) ** 2).sum(axis=1)).max())
                row.append(Box(lo, hi, c, r))
            self.boxes.append(row)
        self.entries_generated = 0

    # -- entries ---------------------------------------------------------
    def _block(self, obs_pts, src_pts, which_rows, which_cols):
        """A(eq rows at obs_pts[e], unknown cols at src_pts[t]) stacked 2x2.

        obs_pts/src_pts are [list_for_half_1, list_for_half_2] of node ids."""
        g = self.g
        out_rows = []
        for e in range(2):
            if len(obs_pts[e]) == 0:
                continue
            blk = []
            for t in range(2):
                if len(src_pts[t]) == 0:
                    continue
                o = PointSet.boundary(g, obs_pts[e])
                s = PointSet.boundary(g, src_pts[t])
                B = system_blocks(o, s, self.med, self.row_scaled, self.eq)[2 * e + t]
                self.entries_generated += B.size
                blk.append(B)
            out_rows.append(np.hstack(blk) if blk else np.zeros((len(obs_pts[e]), 0)))
        return np.vstack(out_rows)

    def _proxy_rows(self, box: Box, cols):
        """M_R: observation = proxy circle + near rows; sources = the box's columns."""
        Rp = self.ratio * box.radius
        npx = proxy_count(self.med.k1, Rp, self.n_proxy_min)
        prox = PointSet.proxy_circle(box.center, Rp, npx)
        near = self._near(box, Rp, rows=True)
        halves = []
        for t in range(2):
            s = PointSet.boundary(self.g, cols[t])
            parts = []
            for e in range(2):
                parts.append(system_blocks(prox, s, self.med, self.row_scaled, self.eq)[2 * e + t])
            for e in range(2):
                if len(near[e]):
                    o = PointSet.boundary(self.g, near[e])
                    parts.append(system_blocks(o, s, self.med, self.row_scaled, self.eq)[2 * e + t])
            M = np.vstack(parts)
            self.entries_generated += M.size
            halves.append(M)
        return halves

    def _proxy_cols_T(self, box: Box, rows):
        """M_L^T: rows = the box's rows, columns = proxy circle + near columns; returned transposed."""
        Rp = self.ratio * box.radius
        npx = proxy_count(self.med.k1, Rp, self.n_proxy_min)
        prox = PointSet.proxy_circle(box.center, Rp, npx)
        near = self._near(box, Rp, rows=False)
        halves = []
        for e in range(2):
            o = PointSet.boundary(self.g, rows[e])
            parts = []
            for t in range(2):
                parts.append(system_blocks(o, prox, self.med, self.row_scaled, self.eq)[2 * e + t])
            for t in range(2):
                if len(near[t]):
                    s = PointSet.boundary(self.g, near[t])
                    parts.append(system_blocks(o, s, self.med, self.row_scaled, self.eq)[2 * e + t])
            M = np.hstack(parts)
            self.entries_generated += M.size
            halves.append(M.T)
        return halves

    def _near(self, box: Box, Rp: float, rows: bool):
        lev = self._cur_level
        out = [[], []]
        for other in self.boxes[lev]:
            if other is box:
                continue
            lists = other.rows if rows else other.cols
            for h in range(2):
                idx = np.asarray(lists[h], dtype=np.int64)
                if idx.size == 0:
                    continue
                d = np.sqrt(((self.g.x[idx] - box.center) ** 2).sum(axis=1))
                out[h].extend(idx[d < Rp].tolist())
        return [np.asarray(o, dtype=np.int64) for o in out]

    # -- compression -----------------------------------------------------
    def compress(self):
        for lev in range(self.L, 0, -1):
            self._cur_level = lev
            for bi, box in enumerate(self.boxes[lev]):
                if lev == self.L:
                    pts = np.arange(box.lo, box.hi)
                    box.rows = [pts, pts]
                    box.cols = [pts, pts]
                else:
                    c1, c2 = self.boxes[lev + 1][2 * bi], self.boxes[lev + 1][2 * bi + 1]
                    box.rows = [np.concatenate([c1.rskel[h], c2.rskel[h]]) for h in range(2)]
                    box.cols = [np.concatenate([c1.cskel[h], c2.cskel[h]]) for h in range(2)]
            rank = self.fixed_rank
            if self.schedule is not None:
                kL, a = self.schedule
                rank = int(round(kL * a ** (self.L - lev)))
            for box in self.boxes[lev]:
                MR = self._proxy_rows(box, box.cols)
                cid = [column_id(MR[h], self.tol, rank) for h in range(2)]
                if self.two_sided:
                    MLt = self._proxy_cols_T(box, box.rows)
                    rid = [column_id(MLt[h], self.tol, rank) for h in range(2)]
                    ks = [max(cid[h][0], rid[h][0]) for h in range(2)]
                    cid = [column_id(MR[h], self.tol, ks[h]) if ks[h] != cid[h][0] else cid[h]
                           for h in range(2)]
                    rid = [column_id(MLt[h], self.tol, ks[h]) if ks[h] != rid[h][0] else rid[h]
                           for h in range(2)]
                else:
                    rid = cid
                box.cskel = [box.cols[h][cid[h][1][:cid[h][0]]] for h in range(2)]
                box.rskel = [box.rows[h][rid[h][1][:rid[h][0]]] for h in range(2)]
                Rq = interp_matrix(cid[0][0], cid[0][1], cid[0][2])
                Ru = interp_matrix(cid[1][0], cid[1][1], cid[1][2])
                box.R = scipy.linalg.block_diag(Rq, Ru)
                Lq = interp_matrix(rid[0][0], rid[0][1], rid[0][2]).T
                Lu = interp_matrix(rid[1][0], rid[1][1], rid[1][2]).T
                box.L = scipy.linalg.block_diag(Lq, Lu)
                box.ranks = (cid[0][0], cid[1][0])

    # -- factorisation -----------------------------------------------------
    def _diag_block(self, lev, bi):
        box = self.boxes[lev][bi]
        D = self._block(box.rows, box.cols, None, None)
        if lev < self.L:
            c1, c2 = self.boxes[lev + 1][2 * bi], self.boxes[lev + 1][2 * bi + 1]
            ri, ci = self._child_index_maps(c1, c2)
            for c, rmap, cmap in ((c1, ri[0], ci[0]), (c2, ri[1], ci[1])):
                D[np.ix_(rmap, cmap)] = c.At
        return D

    @staticmethod
    def _child_index_maps(c1, c2):
        """Positions of each child's compressed unknowns inside the parent's
        [half1: c1, c2; half2: c1, c2] ordering, for rows and for columns."""
        def maps(sk1, sk2):
            n1 = [len(sk1[0]), len(sk1[1])]
            n2 = [len(sk2[0]), len(sk2[1])]
            base2 = n1[0] + n2[0]
            m1 = np.concatenate([np.arange(n1[0]), base2 + np.arange(n1[1])])
            m2 = np.concatenate([n1[0] + np.arange(n2[0]), base2 + n1[1] + np.arange(n2[1])])
            return m1, m2
        return maps(c1.rskel, c2.rskel), maps(c1.cskel, c2.cskel)

    def factor(self):
        for lev in range(self.L, 0, -1):
            for bi, box in enumerate(self.boxes[lev]):
                box.D = self._diag_block(lev, bi)
                box.lu = scipy.linalg.lu_factor(box.D)
                box.X = scipy.linalg.lu_solve(box.lu, box.L)
                box.At = np.linalg.inv(box.R @ box.X)
        root = self.boxes[0][0]
        c1, c2 = self.boxes[1]
        root.rows = [np.concatenate([c1.rskel[h], c2.rskel[h]]) for h in range(2)]
        root.cols = [np.concatenate([c1.cskel[h], c2.cskel[h]]) for h in range(2)]
        root.D = self._diag_block(0, 0)
        root.lu = scipy.linalg.lu_factor(root.D)

    # -- solve -------------------------------------------------------------
    def solve(self, b):
        n = self.g.n
        b = np.asarray(b, dtype=np.complex128)
        f = {}
        g = {}
        ft = {}
        for lev in range(self.L, 0, -1):
            for bi, box in enumerate(self.boxes[lev]):
                if lev == self.L:
                    fb = np.concatenate([b[box.lo:box.hi], b[n + box.lo:n + box.hi]])
                else:
                    fb = self._gather_children(lev, bi, ft)
                f[(lev, bi)] = fb
                g[(lev, bi)] = scipy.linalg.lu_solve(box.lu, fb)
                ft[(lev, bi)] = box.At @ (box.R @ g[(lev, bi)])
        root = self.boxes[0][0]
        y = {(0, 0): scipy.linalg.lu_solve(root.lu, self._gather_children(0, 0, ft))}
        x = np.zeros(2 * n, dtype=np.complex128)
        for lev in range(1, self.L + 1):
            for bi, box in enumerate(self.boxes[lev]):
                yb = self._scatter_to_child(lev, bi, y)
                xb = g[(lev, bi)] - box.X @ (ft[(lev, bi)] - box.At @ yb)
                if lev == self.L:
                    m = box.hi - box.lo
                    x[box.lo:box.hi] = xb[:m]
                    x[n + box.lo:n + box.hi] = xb[m:]
                else:
                    y[(lev, bi)] = xb
        return x

    def _gather_children(self, lev, bi, ft):
        c1, c2 = self.boxes[lev + 1][2 * bi], self.boxes[lev + 1][2 * bi + 1]
        (r1, r2), _ = self._child_index_maps(c1, c2)
        out = np.zeros(len(r1) + len(r2), dtype=np.complex128)
        out[r1] = ft[(lev + 1, 2 * bi)]
        out[r2] = ft[(lev + 1, 2 * bi + 1)]
        return out

    def _scatter_to_child(self, lev, bi, y):
        parent = y[(lev - 1, bi // 2)]
        c1, c2 = self.boxes[lev][2 * (bi // 2)], self.boxes[lev][2 * (bi // 2) + 1]
        _, (m1, m2) = self._child_index_maps(c1, c2)
        return parent[m1] if bi % 2 == 0 else parent[m2]
