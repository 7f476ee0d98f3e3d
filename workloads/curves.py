"""Analytic closed curves sampled at equispaced parameter values.

Every curve is 2*pi-periodic and counter-clockwise, with theta_j = 2*pi*j/N,
j = 0..N-1 (the equispaced trapezoidal nodes of the Nystrom rule, Section 3.1
of the paper).  Each sampler returns three float64 arrays of shape (N, 2):
the point x(theta_j), its derivative x'(theta_j) and second derivative
x''(theta_j).  The derivatives are exact (hand-differentiated), not finite
differences.  ``curve_at`` evaluates the same curves at arbitrary theta.

Shapes:
  circle           x = R (cos t, sin t)
  star(a, m)       r(t) = 1 + a cos(m t),  x = r (cos t, sin t)
  kite             x = (cos t + 0.65 cos 2t - 0.65, 1.5 sin t)   (the
                   Colton-Kress kite; the paper shows a kite only as an image)
"""

from __future__ import annotations

import numpy as np


def _theta(n: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n, dtype=np.float64) / n


def _circle(t, radius: float = 1.0):
    c, s = np.cos(t), np.sin(t)
    return (radius * np.stack([c, s], axis=-1), radius * np.stack([-s, c], axis=-1),
            radius * np.stack([-c, -s], axis=-1))


def _star(t, amp: float = 0.3, arms: int = 5):
    c, s = np.cos(t), np.sin(t)
    r = 1.0 + amp * np.cos(arms * t)
    dr = -amp * arms * np.sin(arms * t)
    ddr = -amp * arms * arms * np.cos(arms * t)
    x = np.stack([r * c, r * s], axis=-1)
    dx = np.stack([dr * c - r * s, dr * s + r * c], axis=-1)
    ddx = np.stack([ddr * c - 2.0 * dr * s - r * c, ddr * s + 2.0 * dr * c - r * s], axis=-1)
    return x, dx, ddx


def _kite(t):
    x = np.stack([np.cos(t) + 0.65 * np.cos(2 * t) - 0.65, 1.5 * np.sin(t)], axis=-1)
    dx = np.stack([-np.sin(t) - 1.3 * np.sin(2 * t), 1.5 * np.cos(t)], axis=-1)
    ddx = np.stack([-np.cos(t) - 2.6 * np.cos(2 * t), -1.5 * np.sin(t)], axis=-1)
    return x, dx, ddx


_CURVES = {"circle": _circle, "star": _star, "kite": _kite}


def curve_at(kind: str, theta, **params):
    """(x, x', x'') at arbitrary parameter values, each shape theta.shape + (2,)."""
    if kind not in _CURVES:
        raise ValueError(f"unknown curve kind {kind!r}")
    return _CURVES[kind](np.asarray(theta, dtype=np.float64), **params)


def sample_curve(kind: str, n: int, **params):
    """Samples at theta_j = 2 pi j / n: 'circle' (radius), 'star' (amp, arms) or 'kite'."""
    return curve_at(kind, _theta(n), **params)


def circle(n: int, radius: float = 1.0):
    return sample_curve("circle", n, radius=radius)


def star(n: int, amp: float = 0.3, arms: int = 5):
    return sample_curve("star", n, amp=amp, arms=arms)


def kite(n: int):
    return sample_curve("kite", n)
