"""Closed forms on the unit circle.

Operator eigenvalues.  On the unit circle every layer operator is a
convolution, so e^{i n theta} is an eigenfunction.  Graf's addition theorem
G_k(x, y) = (i/4) sum_m J_m(k|y|) H_m(k|x|) e^{i m (theta_x - theta_y)}
(|y| < |x|) integrated against e^{i n theta_y} gives
  S_k            : (i pi / 2) J_n(k) H_n(k)
  D_k = D*_k     : (i pi k / 2) J_n(k) H_n'(k) + 1/2   (principal value: the
                   mean of the two one-sided limits; J_n H_n' - J_n' H_n = 2i/(pi k))
  N_k            : (i pi k^2 / 2) J_n'(k) H_n'(k)
for the normal pointing out of the disc.

Transmission solution.  For the problem of Section 2 with a plane wave
u_in = exp(i k0 rho cos(theta - alpha)) = sum_n i^n J_n(k0 rho) e^{i n (theta - alpha)},
write u0_sc = sum a_n H_n(k0 rho) e^{in(theta-alpha)} and
u1_sc = sum b_n J_n(k1 rho) e^{in(theta-alpha)}.  Continuity of u and of
q = (1/eps) d u / d nu on rho = 1 gives per mode
  i^n J_n(k0) + a_n H_n(k0) = b_n J_n(k1)
  (i^n k0 J_n'(k0) + a_n k0 H_n'(k0)) / eps0 = b_n k1 J_n'(k1) / eps1
and on the boundary u = sum b_n J_n(k1) e^{...}, q = sum b_n k1 J_n'(k1) e^{...} / eps1.
"""

from __future__ import annotations

import numpy as np
from scipy import special


def circle_eigs(n: int, k: float):
    """(S, D, N) eigenvalues of mode n on the unit circle."""
    J = special.jv(n, k)
    Jp = special.jvp(n, k)
    H = special.hankel1(n, k)
    Hp = special.h1vp(n, k)
    S = 0.5j * np.pi * J * H
    D = 0.5j * np.pi * k * J * Hp + 0.5
    N = 0.5j * np.pi * k * k * Jp * Hp
    return S, D, N


def circle_transmission(n_nodes: int, k0: float, k1: float, eps0: float, eps1: float,
                        angle: float = 0.0, modes: int | None = None):
    """Boundary values (q, u) of the exact solution at theta_j = 2 pi j / n_nodes."""
    if modes is None:
        modes = int(max(k0, k1) + 60)
    theta = 2.0 * np.pi * np.arange(n_nodes) / n_nodes
    q = np.zeros(n_nodes, dtype=np.complex128)
    u = np.zeros(n_nodes, dtype=np.complex128)
    for n in range(-modes, modes + 1):
        inc = 1j ** (n % 4)
        J0n, J0p = special.jv(n, k0), special.jvp(n, k0)
        H0n, H0p = special.hankel1(n, k0), special.h1vp(n, k0)
        J1n, J1p = special.jv(n, k1), special.jvp(n, k1)
        M = np.array([[H0n, -J1n], [k0 * H0p / eps0, -k1 * J1p / eps1]], dtype=np.complex128)
        rhs = np.array([-inc * J0n, -inc * k0 * J0p / eps0], dtype=np.complex128)
        a, b = np.linalg.solve(M, rhs)
        ph = np.exp(1j * n * (theta - angle))
        u += b * J1n * ph
        q += b * k1 * J1p / eps1 * ph
    return q, u
