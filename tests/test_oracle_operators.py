"""Pins of the oracle's discretised layer operators.

1. Unit circle: each operator applied to e^{i n theta} against the closed-form
   eigenvalue (Graf's addition theorem), converging at third order.
2. The closed-form eigenvalues themselves against direct numerical quadrature.
3. Smooth star: each Nystrom row (with its one-point corrected diagonal)
   against an independent graded Gauss-Legendre quadrature of the continuous
   operator; third-order convergence pins the corrected diagonals
   (Section 3.1), including N_k0 - N_k1.
4. Calderon identities with point sources: for v = G_k(., z),
   z inside the curve: (D_k - W/2) v - S_k dv/dnu = 0 (exterior representation),
   z outside:          (D_k + W/2) v - S_k dv/dnu = 0 (interior representation),
   which fix the free-term signs of eq. symmetric_muller.
"""

import numpy as np
import pytest
from scipy import special

import workloads
from oracle import exact, geometry, kernels
from oracle.kernels import Medium, PointSet


def _circle_errors(n, k0=10.0, k1=15.0, mode=3):
    g = geometry.discretize(*workloads.circle(n))
    S, D, Ds = kernels.single_operators(g, k0)
    Nd = kernels.ndiff_operator(g, k0, k1)
    th = 2 * np.pi * np.arange(n) / n
    v = np.exp(1j * mode * th)
    eS, eD, eN0 = exact.circle_eigs(mode, k0)
    _, _, eN1 = exact.circle_eigs(mode, k1)
    w = g.w
    return np.array([
        np.abs(S @ v / w - eS * v).max() / abs(eS),
        np.abs(D @ v / w - eD * v).max() / abs(eD),
        np.abs(Ds @ v / w - eD * v).max() / abs(eD),
        np.abs(Nd @ v / w - (eN0 - eN1) * v).max() / abs(eN0 - eN1),
    ])


def test_circle_eigenvalues_third_order():
    e = [_circle_errors(n) for n in (64, 128, 256, 512)]
    for a, b in zip(e[:-1], e[1:]):
        assert np.all(a / b > 7.0), (a, b)
    assert np.all(e[-1] < np.array([4e-5, 2e-6, 2e-6, 1e-5]))


def test_circle_eigs_closed_form_vs_quadrature():
    from scipy import integrate
    k, mode = 7.0, 2
    eS, eD, _ = exact.circle_eigs(mode, k)

    def s_int(t, part):
        r = 2.0 * abs(np.sin(t / 2.0))
        val = 0.25j * special.hankel1(0, k * r) * np.exp(1j * mode * t)
        return val.real if part == 0 else val.imag

    def d_int(t, part):
        # x = (1, 0), y = (cos t, sin t), nu_y = y: (x - y).nu_y = cos t - 1
        r = 2.0 * abs(np.sin(t / 2.0))
        val = 0.25j * k * special.hankel1(1, k * r) * (np.cos(t) - 1.0) / r * np.exp(1j * mode * t)
        return val.real if part == 0 else val.imag

    sv = sum(integrate.quad(s_int, a, b, args=(p,), limit=400, epsabs=1e-14, epsrel=1e-13)[0] * (1j if p else 1)
             for (a, b) in ((0, np.pi), (np.pi, 2 * np.pi)) for p in (0, 1))
    dv = sum(integrate.quad(d_int, a, b, args=(p,), limit=400, epsabs=1e-14, epsrel=1e-13)[0] * (1j if p else 1)
             for (a, b) in ((0, np.pi), (np.pi, 2 * np.pi)) for p in (0, 1))
    assert abs(sv - eS) < 1e-11 * abs(eS)
    # the principal value of the double layer on the curve is the eigenvalue
    assert abs(dv - eD) < 1e-11 * abs(eD)


# ---------------------------------------------------------------- star rows
STAR = dict(amp=0.3, arms=5)


def _mp_star(t):
    import mpmath as mp
    a, m = mp.mpf(STAR["amp"]), STAR["arms"]
    c, s = mp.cos(t), mp.sin(t)
    r = 1 + a * mp.cos(m * t)
    dr = -a * m * mp.sin(m * t)
    return (r * c, r * s), (dr * c - r * s, dr * s + r * c)


def _mp_integrand(th_i, t, k0, k1):
    """G_k0, dG/dnu_y, dG/dnu_x, N_k0 - N_k1 (times |y'|) at 30 digits."""
    import mpmath as mp
    (x0, x1), (dx0, dx1) = _mp_star(th_i)
    (y0, y1), (dy0, dy1) = _mp_star(t)
    sx, sy = mp.sqrt(dx0**2 + dx1**2), mp.sqrt(dy0**2 + dy1**2)
    nx, ny = (dx1 / sx, -dx0 / sx), (dy1 / sy, -dy0 / sy)
    d0, d1 = x0 - y0, x1 - y1
    r = mp.sqrt(d0**2 + d1**2)
    dnx, dny = d0 * nx[0] + d1 * nx[1], d0 * ny[0] + d1 * ny[1]
    nn = nx[0] * ny[0] + nx[1] * ny[1]
    out = []
    nk = []
    for k in (k0, k1):
        H0, H1 = mp.hankel1(0, k * r), mp.hankel1(1, k * r)
        ik4 = mp.mpc(0, 1) * k / 4
        if k == k0:
            out += [mp.mpc(0, 1) / 4 * H0, ik4 * H1 * dny / r, -ik4 * H1 * dnx / r]
        nk.append(ik4 * (H1 / r * nn + (k * H0 - 2 * H1 / r) * dnx * dny / r**2))
    out.append(nk[0] - nk[1])
    return np.array([complex(v * sy) for v in out])


def _gl_panels(edges, order):
    x, w = np.polynomial.legendre.leggauss(order)
    ts, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        ts.append(0.5 * (b - a) * x + 0.5 * (b + a))
        ws.append(0.5 * (b - a) * w)
    return np.concatenate(ts), np.concatenate(ws)


def _density(t):
    return np.exp(np.cos(t) + 0.3j * np.sin(2 * t)) * (1.0 + 0.2 * np.cos(3 * t))


def _continuous_rows(th_i, med):
    """(S_k0 phi)(x_i), (D_k0 phi), (D*_k0 phi), ((N_k0 - N_k1) phi) by quadrature.

    Away from the singular point: composite Gauss-Legendre in double precision.
    Within 0.05 of it: panels graded geometrically down to 1e-15, integrand
    at 30 digits (mpmath), so that the log singularity is resolved and the
    N_k0 - N_k1 difference loses nothing to cancellation.
    """
    import mpmath as mp
    s1 = 0.05
    tf, wf = _gl_panels(np.linspace(s1, 2 * np.pi - s1, 65), 16)
    t = th_i + tf
    y, dy, ddy = workloads.curves.curve_at("star", t, **STAR)
    gs = geometry.discretize(y, dy, ddy)
    speed = np.hypot(dy[:, 0], dy[:, 1])
    xi, dxi, ddxi = workloads.curves.curve_at("star", np.array([th_i]), **STAR)
    go = geometry.discretize(xi, dxi, ddxi)
    obs = PointSet(go.x, go.nu, np.ones(1), go.kappa, -np.ones(1, dtype=np.int64))
    src = PointSet(gs.x, gs.nu, np.ones(len(t)), gs.kappa, -np.ones(len(t), dtype=np.int64))
    G0, Dy0, Dx0, N0, _ = kernels.layer_kernels(obs, src, med.k0)
    _, _, _, N1, _ = kernels.layer_kernels(obs, src, med.k1)
    f = _density(t) * speed * wf
    total = np.array([(G0 @ f)[0], (Dy0 @ f)[0], (Dx0 @ f)[0], ((N0 - N1) @ f)[0]])
    tn, wn = _gl_panels(np.concatenate([[0.0], s1 * 2.0 ** -np.arange(50)[::-1]]), 10)
    with mp.workdps(30):
        for sgn in (+1, -1):
            for s, w in zip(tn, wn):
                tt = th_i + sgn * s
                vals = _mp_integrand(mp.mpf(th_i), mp.mpf(th_i) + sgn * mp.mpf(s), med.k0, med.k1)
                total += vals * _density(tt) * w
    return total


def _nystrom_rows(i, n, med):
    g = geometry.discretize(*workloads.star(n, **STAR))
    ps = PointSet.boundary(g)
    obs = ps.take(np.array([i]))
    G0, Dy0, Dx0, N0, same = kernels.layer_kernels(obs, ps, med.k0)
    _, _, _, N1, _ = kernels.layer_kernels(obs, ps, med.k1)
    g0, _, dd, nd = kernels.corrected_diagonals(g.w[i:i + 1], g.kappa[i:i + 1], med)
    Z = [G0[0], Dy0[0], Dx0[0], (N0 - N1)[0]]
    for z, dv in zip(Z, (g0[0], dd[0], dd[0], nd[0])):
        z[i] = dv
    phi = _density(2 * np.pi * np.arange(n) / n) * g.w
    return np.array([z @ phi for z in Z])


@pytest.mark.parametrize("frac", [0.0, 1.0 / 8.0, 37.0 / 128.0])
def test_star_rows_third_order(frac):
    """Rows of S, D, D*, N_k0 - N_k1 with the corrected diagonals: O(h^3)."""
    med = Medium(10.0, 15.0)
    ref = _continuous_rows(2 * np.pi * frac, med)
    errs = []
    for n in (128, 256, 512):
        i = int(round(frac * n))
        errs.append(np.abs(_nystrom_rows(i, n, med) - ref) / np.abs(ref))
    errs = np.array(errs)
    assert np.all(errs[-1] < 5e-5), errs
    assert np.all(errs[0] / errs[-1] > 30.0), errs  # two doublings at third order: ~64


def test_calderon_point_sources_star():
    """Free-term signs and S/D consistency on a non-symmetric-looking curve."""
    res = []
    for n in (128, 256, 512):
        g = geometry.discretize(*workloads.star(n, **STAR))
        row = []
        for k in (10.0, 15.0):
            S, D, _ = kernels.single_operators(g, k)
            for z, sign in (((0.1, -0.2), -1.0), ((1.9, 1.2), +1.0)):
                d = g.x - np.asarray(z)
                r = np.hypot(d[:, 0], d[:, 1])
                v = 0.25j * special.hankel1(0, k * r)
                dv = -0.25j * k * special.hankel1(1, k * r) * (d * g.nu).sum(1) / r
                lhs = D @ v + sign * 0.5 * g.w * v - S @ dv
                row.append(np.linalg.norm(lhs) / np.linalg.norm(g.w * v))
        res.append(row)
    res = np.array(res)
    assert np.all(res[-1] < 2e-4), res
    assert np.all(res[0] / res[-1] > 30.0), res
