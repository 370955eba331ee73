"""Sphere radius selection (Sec. II, radius discussion).

Test infrastructure only (see oracle/__init__.py).

Sec. II names three ways to choose the radius r_c of the atomic spheres:
the cutoff radius of the non-local pseudopotential (no pseudopotentials
here: that radius is the caller's r_c), the smallest dimension of the
simulation cell, and the radius at which the radial part of the orbital
drops below a threshold.

Readings (the paper gives no formulas):
* the smallest dimension of the cell is the shortest cell edge, min_i a_i
  (orthorhombic cells), so a sphere may reach its own periodic images;
* the radial part is the continuum-normalized Slater function
  R(r) = N r^l exp(-zeta r), N = sqrt((2 zeta)^(2l+3) / (2l+2)!), so that
  int_0^inf R^2 r^2 dr = 1; r_c is the radius beyond which R stays below the
  threshold: the root of R(r) = t on r >= l / zeta (where R peaks).  For
  l = 0 it is ln(N / t) / zeta; for l >= 1 it follows from the lower branch
  of the Lambert W function,
      r_c = -(l / zeta) W_{-1}(-(zeta / l) (t / N)^(1/l)).
  A threshold at or above the peak value has no such radius (error).
"""

import math

import numpy as np
from scipy.special import lambertw


def radial_norm(l, zeta):
    return math.sqrt((2.0 * zeta) ** (2 * l + 3) / math.factorial(2 * l + 2))


def radial(l, zeta, r):
    return radial_norm(l, zeta) * np.asarray(r, dtype=np.float64) ** l * np.exp(-zeta * np.asarray(r))


def radius_cell(cell):
    return float(np.min(np.asarray(cell, dtype=np.float64)))


def radius_threshold(l, zeta, threshold):
    N = radial_norm(l, zeta)
    peak = radial(l, zeta, l / zeta) if l > 0 else N
    if not (0.0 < threshold < peak):
        raise ValueError("threshold must lie between 0 and the peak of the radial function")
    if l == 0:
        return math.log(N / threshold) / zeta
    x = -(zeta / l) * (threshold / N) ** (1.0 / l)
    return float(-(l / zeta) * lambertw(x, -1).real)
