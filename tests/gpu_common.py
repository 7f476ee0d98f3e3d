"""Helpers shared by the GPU tests: solver setup and oracle references."""

import numpy as np

import workloads
from oracle import dense, geometry, kernels
from oracle.kernels import Medium


def make_solver(wl, form=0, leaf=None, tol=None, n_proxy=None, root_max=0):
    from paper_2609_33216_amd import binding
    x, dx, ddx = wl.boundary()
    s = binding.Solver(0)
    s.assemble(x, dx, ddx, wl.k0, wl.k1, wl.eps0, wl.eps1, leaf=leaf or wl.leaf, tol=tol or wl.tol, form=form,
               n_proxy=n_proxy or (wl.n_proxy if wl.n_proxy > 0 else 64), proxy_ratio=wl.proxy_ratio,
               root_max=root_max)
    return s


def oracle_system(wl, row_scaled=True, eq="muller"):
    x, dx, ddx = wl.boundary()
    g = geometry.discretize(x, dx, ddx)
    med = Medium(wl.k0, wl.k1, wl.eps0, wl.eps1)
    A = kernels.assemble(g, med, row_scaled, eq)
    uin, qin = dense.plane_wave(g, wl.k0, wl.angle)
    b = dense.rhs(g, med, uin, qin, row_scaled, eq)
    return g, med, A, b


# form of the C-ABI -> (system, row-scaled) of the oracle
FORMS = {0: ("muller", True), 1: ("muller", False), 2: ("muller", True), 3: ("pmchwt", True),
         4: ("pmchwt", False), 5: ("bm", False)}


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
