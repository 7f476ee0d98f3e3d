"""Layer-potential kernels and the Muller-like 2x2 block system, in FP64.

Kernels (Section 3.1, d = x - y, r = |d|, H_n = H_n^(1)):
  G_k(x, y)                  = (i/4) H0(k r)
  dG/dnu(y)   (double layer) = (i k / 4) H1(k r) (d . nu_y) / r
  dG/dnu(x)   (adjoint)      = -(i k / 4) H1(k r) (d . nu_x) / r
  d2G/dnu(x)dnu(y)           = (i k / 4) [ H1(k r)/r (nu_x . nu_y)
                                 + (k H0(k r) - 2 H1(k r)/r) (d.nu_x)(d.nu_y)/r^2 ]
The last one follows from H0' = -H1 and H1'(z) = H0(z) - H1(z)/z.  The
paper's kernel tables write nu(x_j) where the observation normal nu(x_i) is
meant; this module reads nu(x_i).

One-point corrected diagonal (paper Section 3.1: only the i = j entry is
replaced; the paper cites the zeta-corrected rule without printing the
terms).  A kernel f(x_i, y) = a ln|x_i - y| + b + o(1) near y = x_i gets the
diagonal value a*ln(w_i / 2 pi) + b: the punctured trapezoidal rule on
ln|2 sin(t/2)| g(t) misses exactly h g(0) ln(h / 2 pi), and splitting
ln|x_i - y(t)| = ln|t - t_i| + ln|x'_i| + (smooth, zero at t_i) gives
ln(h/2pi) + ln|x'_i| = ln(w_i/2pi).  The small-argument expansions
  G_k        = -(1/2pi) ln r + i/4 - (1/2pi)(ln(k/2) + gamma) + O(r^2 ln r)
  dG/dnu     -> -kappa/(4 pi)                (no logarithm: (d.nu)/r^2 -> -kappa/2)
  N_k0-N_k1  = -(Delta/4pi) ln r + i Delta/8 - (Delta/4pi)(gamma - 1/2)
               - (1/4pi)(k0^2 ln(k0/2) - k1^2 ln(k1/2)) + O(r^2 ln r),
  Delta = k0^2 - k1^2,
give the corrected diagonals below.

The individual N_k (needed by the PMCHWT and Burton-Miller systems) is
hypersingular.  Along the curve, in the parameter t around t_i, its kernel
times |y'| is A/t^2 + C ln|t| + (smooth), A = 1/(2 pi |x'_i|), with no 1/t
term (the Laplace part 1/(2 pi s^2) + kappa^2/(24 pi) in arclength s, pulled
back, gains only a constant).  The punctured trapezoidal sum of
phi(t)/t^2 exceeds the finite-part integral by 2 zeta(2) phi(0)/h -
(h/2) phi''(0) + O(h^3): the one-point rule removes the first term and keeps
the second, which is why N_k converges at first order only (Section 3.1,
estimate for N_k).  The diagonal is
  N~_k = -pi/(6 w_i^2) + kappa_i^2/(24 pi) + i k^2/8
         - (k^2/4pi)(ln(k/2) + gamma - 1/2 + ln(w_i/2pi)),
from N_k = 1/(2 pi r^2) + kappa^2/(24 pi) - (k^2/4pi) ln r + i k^2/8
- (k^2/4pi)(ln(k/2) + gamma - 1/2) + o(1); the difference of two such
diagonals is the N_k0 - N_k1 value above.  A constant that depends on how
the parameter runs along the curve (the Schwarzian derivative of the
arclength, which needs the third derivative of the curve) is left out: it
weighs O(h), as does the rule's own error.

System (eq. symmetric_muller, block form eq. block_A), unknowns [q; u]:
  A11 = -(eps0^2 S_k0 - eps1^2 S_k1)
  A12 = eps0 (D_k0 - W/2) - eps1 (D_k1 + W/2)
  A21 = eps0 (D*_k0 + W/2) - eps1 (D*_k1 - W/2)
  A22 = -(N_k0 - N_k1)
with row-scaled operators [Z]_ij = w_i Z~(x_i, y_j) w_j.  The unscaled
baseline (eq. naive_muller) uses [Z']_ij = Z~(x_i, y_j) w_j and free terms
-/+ (eps0 + eps1)/2 I.  Entries are formed as (w_i w_j) * K so that the
scaled matrix is symmetric up to the free terms to the last bit.

PMCHWT (eq. naive_pmchwt, row-scaled: eq. symmetric_pmchwt), same unknowns:
  A11 = -(eps0 S_k0 + eps1 S_k1)    A12 = D_k0 + D_k1
  A21 = D*_k0 + D*_k1               A22 = -(N_k0 / eps0 + N_k1 / eps1)
(the free terms cancel, so the row-scaled matrix is exactly symmetric).

Burton-Miller (eq. bm), alpha = i / k0.  The paper orders the unknowns
[u; q]; here the columns are permuted to [q; u] so that every system shares
one layout (rows: combined exterior equation, interior equation):
  A11 = -eps0 (S_k0 + alpha (D*_k0 + I/2))   A12 = D_k0 - I/2 + alpha N_k0
  A21 = -eps1 S_k1                           A22 = D_k1 + I/2
The printed system carries +alpha eps0 (D*_k0 + I/2): with the exterior
equations (D_k0 - I/2) u - eps0 S_k0 q = -u_in and
eps0 (D*_k0 + I/2) q - N_k0 u = q_in (the second rows of eq. naive_muller),
only the combination exterior - alpha * (normal derivative) reproduces both
the printed +alpha N_k0 and the printed right-hand side -u_in - alpha q_in,
and that combination has -alpha eps0 (D*_k0 + I/2).  This module takes that
reading (one sign); the printed sign does not converge to the transmission
solution (pinned in the tests).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import bessel
from .geometry import Geometry

EULER_GAMMA = 0.57721566490153286060651209008240243


@dataclasses.dataclass(frozen=True)
class Medium:
    k0: float
    k1: float
    eps0: float = 1.0
    eps1: float = 1.0


@dataclasses.dataclass
class PointSet:
    """Observation or source points: coordinates, unit normals, weights.

    gid holds the boundary index of each point, or -1 for a point that is not
    a boundary node (a proxy point); equal non-negative gids mark the
    diagonal pair that takes the corrected value.
    """
    x: np.ndarray
    nu: np.ndarray
    w: np.ndarray
    kappa: np.ndarray
    gid: np.ndarray

    @staticmethod
    def boundary(geom: Geometry, idx=None) -> "PointSet":
        idx = np.arange(geom.n) if idx is None else np.asarray(idx, dtype=np.int64)
        return PointSet(geom.x[idx], geom.nu[idx], geom.w[idx], geom.kappa[idx], idx.copy())

    @staticmethod
    def proxy_circle(center, radius: float, count: int) -> "PointSet":
        """count equispaced points on a circle, outward normals, weights 2 pi R / count."""
        phi = 2.0 * np.pi * np.arange(count) / count
        nu = np.stack([np.cos(phi), np.sin(phi)], axis=1)
        x = np.asarray(center, dtype=np.float64)[None, :] + radius * nu
        w = np.full(count, 2.0 * np.pi * radius / count)
        return PointSet(x, nu, w, np.zeros(count), -np.ones(count, dtype=np.int64))

    def __len__(self):
        return self.x.shape[0]

    def concat(self, other: "PointSet") -> "PointSet":
        return PointSet(np.concatenate([self.x, other.x]), np.concatenate([self.nu, other.nu]),
                        np.concatenate([self.w, other.w]),
                        np.concatenate([self.kappa, other.kappa]),
                        np.concatenate([self.gid, other.gid]))

    def take(self, sel) -> "PointSet":
        return PointSet(self.x[sel], self.nu[sel], self.w[sel], self.kappa[sel], self.gid[sel])


def layer_kernels(obs: PointSet, src: PointSet, k: float):
    """Off-diagonal kernel values G, dG/dnu_y, dG/dnu_x, d2G/dnu_x dnu_y.

    Pairs with r = 0 (the diagonal) come back as NaN-free placeholders and
    must be overwritten by the caller.
    """
    d0 = obs.x[:, None, 0] - src.x[None, :, 0]
    d1 = obs.x[:, None, 1] - src.x[None, :, 1]
    r = np.hypot(d0, d1)
    same = r == 0.0
    r = np.where(same, 1.0, r)
    z = k * r
    H0 = bessel.h0(z)
    H1 = bessel.h1(z)
    dny = d0 * src.nu[None, :, 0] + d1 * src.nu[None, :, 1]
    dnx = d0 * obs.nu[:, None, 0] + d1 * obs.nu[:, None, 1]
    nxny = obs.nu[:, None, 0] * src.nu[None, :, 0] + obs.nu[:, None, 1] * src.nu[None, :, 1]
    ik4 = 0.25j * k
    G = 0.25j * H0
    Dy = ik4 * H1 * dny / r
    Dx = (-ik4) * H1 * dnx / r
    Nk = ik4 * (H1 / r * nxny + (k * H0 - 2.0 * H1 / r) * (dnx * dny) / (r * r))
    return G, Dy, Dx, Nk, same


def corrected_diagonals(w, kappa, med: Medium):
    """One-point corrected diagonal kernel values for the two wavenumbers.

    Returns (G0~, G1~, D~, ND~) per point: G~ for k0 and k1, the double-layer
    (and adjoint) diagonal -kappa/(4 pi) (wavenumber independent) and the
    diagonal of N_k0 - N_k1.
    """
    ell = np.log(np.asarray(w) / (2.0 * np.pi))
    k0, k1 = med.k0, med.k1
    g = EULER_GAMMA

    def gdiag(k):
        return 0.25j - (np.log(k / 2.0) + g + ell) / (2.0 * np.pi)

    dd = -np.asarray(kappa) / (4.0 * np.pi)
    delta = k0 * k0 - k1 * k1
    nd = (0.125j * delta - (2.0 * g - 1.0) / (8.0 * np.pi) * delta
          - (k0 * k0 * np.log(k0 / 2.0) - k1 * k1 * np.log(k1 / 2.0)) / (4.0 * np.pi)
          - delta / (4.0 * np.pi) * ell)
    return gdiag(k0), gdiag(k1), dd, nd


def n_single_diagonal(w, kappa, k: float):
    """One-point corrected diagonal of the hypersingular N_k (see module text)."""
    w = np.asarray(w, dtype=np.float64)
    ell = np.log(w / (2.0 * np.pi))
    kap = np.asarray(kappa, dtype=np.float64)
    return (-np.pi / (6.0 * w * w) + kap * kap / (24.0 * np.pi) + 0.125j * k * k
            - k * k / (4.0 * np.pi) * (np.log(k / 2.0) + EULER_GAMMA - 0.5 + ell))


def _diag_pairs(obs: PointSet, src: PointSet, same):
    diag = (obs.gid[:, None] == src.gid[None, :]) & (obs.gid[:, None] >= 0)
    if np.any(same & ~diag):
        raise ValueError("coincident points that are not the same boundary node")
    return np.nonzero(diag)


def _weights(obs: PointSet, src: PointSet, shape, row_scaled: bool):
    if row_scaled:
        return obs.w[:, None] * src.w[None, :]
    return np.broadcast_to(src.w[None, :], shape)


def pmchwt_blocks(obs: PointSet, src: PointSet, med: Medium, row_scaled: bool = True):
    """A11, A12, A21, A22 of eq. symmetric_pmchwt (row-scaled) or eq. naive_pmchwt."""
    e0, e1 = med.eps0, med.eps1
    G0, Dy0, Dx0, N0, same = layer_kernels(obs, src, med.k0)
    G1, Dy1, Dx1, N1, _ = layer_kernels(obs, src, med.k1)
    K11 = -(e0 * G0 + e1 * G1)
    K12 = Dy0 + Dy1
    K21 = Dx0 + Dx1
    K22 = -(N0 / e0 + N1 / e1)
    io, js = _diag_pairs(obs, src, same)
    if len(io):
        g0, g1, dd, _ = corrected_diagonals(obs.w[io], obs.kappa[io], med)
        n0 = n_single_diagonal(obs.w[io], obs.kappa[io], med.k0)
        n1 = n_single_diagonal(obs.w[io], obs.kappa[io], med.k1)
        K11[io, js] = -(e0 * g0 + e1 * g1)
        K12[io, js] = dd + dd
        K21[io, js] = dd + dd
        K22[io, js] = -(n0 / e0 + n1 / e1)
    ww = _weights(obs, src, K11.shape, row_scaled)
    return ww * K11, ww * K12, ww * K21, ww * K22


def bm_alpha(med: Medium) -> complex:
    """Burton-Miller coupling constant alpha = i / k0 (Section 6.1)."""
    return 1j / med.k0


def bm_blocks(obs: PointSet, src: PointSet, med: Medium, row_scaled: bool = False):
    """A11, A12, A21, A22 of eq. bm with the columns in [q; u] order.

    row_scaled=False is the printed (unscaled) system; True multiplies each
    row by w_i (same solution)."""
    e0, e1 = med.eps0, med.eps1
    al = bm_alpha(med)
    G0, Dy0, Dx0, N0, same = layer_kernels(obs, src, med.k0)
    G1, Dy1, _, _, _ = layer_kernels(obs, src, med.k1)
    K11 = -e0 * (G0 + al * Dx0)
    K12 = Dy0 + al * N0
    K21 = -e1 * G1
    K22 = Dy1.copy()
    io, js = _diag_pairs(obs, src, same)
    free = np.zeros(len(io))
    if len(io):
        g0, g1, dd, _ = corrected_diagonals(obs.w[io], obs.kappa[io], med)
        n0 = n_single_diagonal(obs.w[io], obs.kappa[io], med.k0)
        K11[io, js] = -e0 * (g0 + al * dd)
        K12[io, js] = dd + al * n0
        K21[io, js] = -e1 * g1
        K22[io, js] = dd
        free = 0.5 * (obs.w[io] if row_scaled else np.ones(len(io)))
    ww = _weights(obs, src, K11.shape, row_scaled)
    A11, A12, A21, A22 = ww * K11, ww * K12, ww * K21, ww * K22
    if len(io):
        A11[io, js] -= al * e0 * free
        A12[io, js] -= free
        A22[io, js] += free
    return A11, A12, A21, A22


EQUATIONS = ("muller", "pmchwt", "bm")


def system_blocks(obs: PointSet, src: PointSet, med: Medium, row_scaled: bool = True, eq: str = "muller"):
    """The four sub-blocks of the chosen system between obs and src points."""
    if eq == "muller":
        return muller_blocks(obs, src, med, row_scaled)
    if eq == "pmchwt":
        return pmchwt_blocks(obs, src, med, row_scaled)
    if eq == "bm":
        return bm_blocks(obs, src, med, row_scaled)
    raise ValueError(f"unknown system {eq!r}")


def muller_blocks(obs: PointSet, src: PointSet, med: Medium, row_scaled: bool = True):
    """The four sub-blocks A11, A12, A21, A22 between obs and src points.

    row_scaled=True gives eq. symmetric_muller entries w_o K w_s,
    False gives eq. naive_muller entries K w_s.  Diagonal pairs (same
    boundary index) take the corrected kernel and the free terms.
    """
    e0, e1 = med.eps0, med.eps1
    G0, Dy0, Dx0, N0, same = layer_kernels(obs, src, med.k0)
    G1, Dy1, Dx1, N1, _ = layer_kernels(obs, src, med.k1)
    K11 = -(e0 * e0 * G0 - e1 * e1 * G1)
    K12 = e0 * Dy0 - e1 * Dy1
    K21 = e0 * Dx0 - e1 * Dx1
    K22 = -(N0 - N1)

    diag = (obs.gid[:, None] == src.gid[None, :]) & (obs.gid[:, None] >= 0)
    if np.any(same & ~diag):
        raise ValueError("coincident points that are not the same boundary node")
    io, js = np.nonzero(diag)
    free = np.zeros(len(io))
    if len(io):
        g0, g1, dd, nd = corrected_diagonals(obs.w[io], obs.kappa[io], med)
        K11[io, js] = -(e0 * e0 * g0 - e1 * e1 * g1)
        K12[io, js] = (e0 - e1) * dd
        K21[io, js] = (e0 - e1) * dd
        K22[io, js] = -nd
        free = 0.5 * (e0 + e1) * (obs.w[io] if row_scaled else np.ones(len(io)))

    if row_scaled:
        ww = obs.w[:, None] * src.w[None, :]
    else:
        ww = np.broadcast_to(src.w[None, :], K11.shape)
    A11 = ww * K11
    A12 = ww * K12
    A21 = ww * K21
    A22 = ww * K22
    if len(io):
        A12[io, js] -= free
        A21[io, js] += free
    return A11, A12, A21, A22


def assemble(geom: Geometry, med: Medium, row_scaled: bool = True, eq: str = "muller") -> np.ndarray:
    """Dense 2N x 2N matrix in the paper's block order [q; u]."""
    ps = PointSet.boundary(geom)
    A11, A12, A21, A22 = system_blocks(ps, ps, med, row_scaled, eq)
    return np.block([[A11, A12], [A21, A22]])


def entries(geom: Geometry, med: Medium, rows, cols, row_scaled: bool = True, eq: str = "muller") -> np.ndarray:
    """A[rows][:, cols] of the 2N x 2N system without forming all of A.

    rows/cols index the unknowns: i < N is the q-equation / q-unknown of node
    i, N + i the u-equation / u-unknown of node i.
    """
    n = geom.n
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    rp, rb = rows % n, rows // n
    cp, cb = cols % n, cols // n
    blocks = system_blocks(PointSet.boundary(geom, rp), PointSet.boundary(geom, cp), med, row_scaled, eq)
    out = np.empty((len(rows), len(cols)), dtype=np.complex128)
    for bi in (0, 1):
        for bj in (0, 1):
            m = (rb[:, None] == bi) & (cb[None, :] == bj)
            out[m] = blocks[2 * bi + bj][m]
    return out


def single_operators(geom: Geometry, k: float, row_scaled: bool = True):
    """Row-scaled S_k, D_k, D*_k and the corrected-diagonal of each (no N_k).

    Used to check the operators one at a time against closed forms and the
    symmetric relations S = S^T, D = D*^T.
    """
    ps = PointSet.boundary(geom)
    G, Dy, Dx, _, _ = layer_kernels(ps, ps, k)
    med = Medium(k, k)
    g, _, dd, _ = corrected_diagonals(geom.w, geom.kappa, med)
    i = np.arange(geom.n)
    G[i, i] = g
    Dy[i, i] = dd
    Dx[i, i] = dd
    ww = geom.w[:, None] * geom.w[None, :] if row_scaled else np.broadcast_to(geom.w[None, :], G.shape)
    return ww * G, ww * Dy, ww * Dx


def ndiff_operator(geom: Geometry, k0: float, k1: float, row_scaled: bool = True):
    """(N_k0 - N_k1) with the corrected diagonal, row-scaled or not."""
    ps = PointSet.boundary(geom)
    _, _, _, N0, _ = layer_kernels(ps, ps, k0)
    _, _, _, N1, _ = layer_kernels(ps, ps, k1)
    Z = N0 - N1
    _, _, _, nd = corrected_diagonals(geom.w, geom.kappa, Medium(k0, k1))
    i = np.arange(geom.n)
    Z[i, i] = nd
    ww = geom.w[:, None] * geom.w[None, :] if row_scaled else np.broadcast_to(geom.w[None, :], Z.shape)
    return ww * Z


def n_single_operator(geom: Geometry, k: float, row_scaled: bool = True):
    """The hypersingular N_k with its one-point corrected diagonal."""
    ps = PointSet.boundary(geom)
    _, _, _, Z, _ = layer_kernels(ps, ps, k)
    i = np.arange(geom.n)
    Z[i, i] = n_single_diagonal(geom.w, geom.kappa, k)
    ww = geom.w[:, None] * geom.w[None, :] if row_scaled else np.broadcast_to(geom.w[None, :], Z.shape)
    return ww * Z
