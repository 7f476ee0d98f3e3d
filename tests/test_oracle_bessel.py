"""Pins of the oracle's Hankel functions (SciPy/AMOS) against mpmath.

mpmath evaluates J and Y at 40 significant digits by its own series and
asymptotic code, independent of AMOS.  The Wronskian J1 Y0 - J0 Y1 = 2/(pi z)
(DLMF 10.5.2) is a second, library-free check.
"""

import mpmath
import numpy as np
import pytest

from oracle import bessel

Z = np.concatenate([np.geomspace(1e-4, 2e3, 61), [2.404825557695773, 3.8317059702075125, 8.0, 25.0]])


def _mp(z):
    with mpmath.workdps(40):
        return (complex(mpmath.hankel1(0, z)), complex(mpmath.hankel1(1, z)))


@pytest.mark.parametrize("z", Z)
def test_hankel_vs_mpmath(z):
    h0m, h1m = _mp(z)
    h0, h1 = complex(bessel.h0(z)), complex(bessel.h1(z))
    # relative to |H|, which has no zeros on the positive axis
    assert abs(h0 - h0m) <= 4e-15 * abs(h0m) + 1e-300
    assert abs(h1 - h1m) <= 4e-15 * abs(h1m) + 1e-300


def test_wronskian():
    j0, y0, j1, y1 = bessel.jy01(Z)
    w = j1 * y0 - j0 * y1
    scale = np.sqrt((j0**2 + y0**2) * (j1**2 + y1**2))
    assert np.all(np.abs(w - 2.0 / (np.pi * Z)) <= 1e-14 * np.maximum(scale, 2.0 / (np.pi * Z)))


def test_small_argument_limits():
    # H0 ~ 1 + (2i/pi)(ln(z/2) + gamma), H1 ~ -2i/(pi z) as z -> 0 (DLMF 10.7.2, 10.7.7)
    z = 1e-6
    g = 0.5772156649015329
    assert abs(bessel.h0(z) - (1 + 2j / np.pi * (np.log(z / 2) + g))) < 1e-10
    assert abs(bessel.h1(z) * (np.pi * z / -2j) - 1.0) < 1e-10
