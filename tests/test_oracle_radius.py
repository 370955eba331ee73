"""Pins for oracle.radius: sphere radius selection (Sec. II).

* The radial function is normalized: int R^2 r^2 dr = 1 by adaptive
  quadrature (not the factorial closed form).
* The threshold radius solves R(r_c) = t to rounding, lies beyond the peak,
  and R stays below t on a fine grid past it; for l = 0 it equals
  ln(N/t)/zeta; for l >= 1 it matches a bracketing root finder (brentq) on
  the log form.
* Thresholds at or above the peak are rejected; smaller thresholds give
  larger radii.
* The cell method is the shortest edge.
"""

import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

from oracle import radius as RA


@pytest.mark.parametrize("l,zeta", [(0, 1.0), (1, 1.6), (2, 2.2), (3, 2.4)])
def test_radial_normalization(l, zeta):
    val, err = quad(lambda r: RA.radial(l, zeta, r) ** 2 * r * r, 0.0, np.inf, epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-10


@pytest.mark.parametrize("l,zeta,t", [(0, 1.0, 1e-3), (1, 1.6, 1e-2), (2, 2.2, 5e-3), (2, 2.2, 1e-4), (3, 2.4, 1e-3)])
def test_threshold_radius(l, zeta, t):
    rc = RA.radius_threshold(l, zeta, t)
    assert rc > l / zeta
    assert abs(RA.radial(l, zeta, rc) - t) < 1e-12 * t * max(1.0, rc * zeta)
    r = np.linspace(rc * (1 + 1e-9), rc + 20.0, 20001)
    assert np.all(RA.radial(l, zeta, r) < t)
    N = RA.radial_norm(l, zeta)
    if l == 0:
        assert abs(rc - math.log(N / t) / zeta) < 1e-13 * rc
    else:
        f = lambda x: math.log(N) + l * math.log(x) - zeta * x - math.log(t)  # noqa: E731
        ref = brentq(f, l / zeta, 200.0, xtol=1e-15, rtol=1e-15)
        assert abs(rc - ref) < 1e-12 * rc
    assert RA.radius_threshold(l, zeta, t / 10) > rc


def test_threshold_out_of_range():
    with pytest.raises(ValueError):
        RA.radius_threshold(2, 2.2, 1.0)
    with pytest.raises(ValueError):
        RA.radius_threshold(0, 1.0, 0.0)


def test_cell_radius():
    assert RA.radius_cell([8.35, 7.1, 9.0]) == 7.1
