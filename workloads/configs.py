"""The measured workloads, as plain seeded descriptions.

Material reading: the paper fixes k_i = omega*sqrt(eps_i) and uses eps_0 = 1
(Section 6).  A workload is quoted by its two wavenumbers, so eps_0 = 1,
omega = k_out and eps_1 = (k_in/k_out)**2.

Incidence: plane wave exp(i k0 (cos(alpha) x1 + sin(alpha) x2)); alpha = 0
travels along x1 as in the paper's experiments.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from .curves import sample_curve


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    curve: str
    curve_params: tuple  # tuple of (key, value) pairs, hashable
    n: int               # boundary points (2n unknowns)
    k0: float            # exterior wavenumber
    k1: float            # interior wavenumber
    angle: float         # plane-wave direction
    leaf: int = 128      # points per HSS leaf
    tol: float = 1e-10   # relative ID tolerance
    n_proxy: int = 0     # proxy points per circle; 0 = size from k*R_p
    proxy_ratio: float = 1.5

    @property
    def eps0(self) -> float:
        return 1.0

    @property
    def eps1(self) -> float:
        return (self.k1 / self.k0) ** 2

    def params(self) -> dict:
        return dict(self.curve_params)

    def boundary(self):
        """(x, dx, ddx), each float64 (n, 2)."""
        return sample_curve(self.curve, self.n, **self.params())

    def with_n(self, n: int, leaf: int | None = None) -> "Workload":
        return dataclasses.replace(self, n=n, leaf=self.leaf if leaf is None else leaf)


def config1() -> Workload:
    """Unit circle, N=2048, k=10/15, angle 0, leaf 64, tol 1e-10, 64 proxies."""
    return Workload("circle-n2048-k10-15", "circle", (), 2048, 10.0, 15.0, 0.0,
                    leaf=64, tol=1e-10, n_proxy=64)


def _angle(seed: int) -> float:
    return float(np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi))


def config2() -> Workload:
    """Five-arm star r = 1 + 0.3 cos 5t, N=32768, k=50/75, leaf 128, tol 1e-10."""
    return Workload("star5-n32768-k50-75", "star", (("amp", 0.3), ("arms", 5)),
                    32768, 50.0, 75.0, _angle(2), leaf=128, tol=1e-10)


def config2_reduced(n: int = 8192) -> Workload:
    """Same curve and wavenumbers as config2 at a size the dense oracle can solve."""
    return dataclasses.replace(config2(), name=f"star5-n{n}-k50-75", n=n)


def config4() -> Workload:
    """Seven-arm star r = 1 + 0.25 cos 7t, N=262144, k=200/300, leaf 128."""
    return Workload("star7-n262144-k200-300", "star", (("amp", 0.25), ("arms", 7)),
                    262144, 200.0, 300.0, _angle(4), leaf=128, tol=1e-10)


def config3_batch(seed: int = 3, count: int = 64, leaf: int = 128, tol: float = 1e-10):
    """Batch of seeded random stars: arms 3..8, amp U[0.1,0.3],
    N log-uniform in [4096, 65536], k_out U[5,80], k_in = 1.5 k_out."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        arms = int(rng.integers(3, 9))
        amp = float(rng.uniform(0.1, 0.3))
        n = int(round(math.exp(rng.uniform(math.log(4096), math.log(65536)))))
        k0 = float(rng.uniform(5.0, 80.0))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        out.append(Workload(f"batch{seed}-{i}", "star", (("amp", amp), ("arms", arms)),
                            n, k0, 1.5 * k0, ang, leaf=leaf, tol=tol))
    return out


def scaled_config(base: Workload, n: int, leaf: int | None = None) -> Workload:
    """Same curve, wavenumbers and settings at another size."""
    return dataclasses.replace(base, name=f"{base.name}@n{n}", n=n,
                               leaf=base.leaf if leaf is None else leaf)
