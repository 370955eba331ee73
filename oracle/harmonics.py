"""Real spherical and solid harmonics for the oracle.

The paper represents each localized orbital as a radial function times a
spherical harmonic (Sec. II, discussion of pseudo-wavefunctions).  The oracle
builds the *real* harmonics from scipy's complex ``sph_harm_y`` (which carries
the Condon-Shortley phase) with the textbook real combination

    m > 0 : sqrt(2) (-1)^m Re Y_l^m
    m = 0 : Y_l^0
    m < 0 : sqrt(2) (-1)^m Im Y_l^{|m|}

so that, for every l, the order m = -l..l gives the standard positive real
harmonics (p: y, z, x).  The solid harmonic is S_lm(r) = |r|^l Y_lm(r_hat), a
homogeneous polynomial of degree l.  Its gradient is obtained from the
polynomial's monomial coefficients, which are recovered here by an exact
linear solve on sample points (no hand-typed derivative table).
"""

import itertools

import numpy as np
from scipy.special import sph_harm_y


def real_ylm(l, m, x, y, z):
    """Real spherical harmonic Y_lm at direction (x, y, z) (any length > 0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r = np.sqrt(x * x + y * y + z * z)
    safe = np.where(r > 0, r, 1.0)
    theta = np.arccos(np.clip(z / safe, -1.0, 1.0))
    phi = np.arctan2(y, x)
    am = abs(m)
    y_c = sph_harm_y(l, am, theta, phi)
    if m > 0:
        val = np.sqrt(2.0) * (-1.0) ** m * y_c.real
    elif m == 0:
        val = y_c.real
    else:
        val = np.sqrt(2.0) * (-1.0) ** m * y_c.imag
    if l == 0:
        return np.broadcast_to(val, r.shape).astype(np.float64).copy()
    return np.where(r > 0, val, 0.0)


def solid_harmonic(l, m, x, y, z):
    """S_lm(r) = |r|^l Y_lm(r_hat); zero at the origin for l >= 1."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r = np.sqrt(x * x + y * y + z * z)
    return r ** l * real_ylm(l, m, x, y, z)


def _monomials(l):
    return [e for e in itertools.product(range(l + 1), repeat=3) if sum(e) == l]


_POLY_CACHE = {}


def solid_harmonic_poly(l, m):
    """Monomial expansion of S_lm: list of ((a, b, c), coeff) with a+b+c = l.

    Recovered by solving the square-or-overdetermined system S(p_i) =
    sum_k coeff_k x_i^a y_i^b z_i^c on seeded random points; the residual is
    checked so that a wrong harmonic can never silently pass.
    """
    key = (l, m)
    if key in _POLY_CACHE:
        return _POLY_CACHE[key]
    mons = _monomials(l)
    rng = np.random.default_rng(1234 + 17 * l + m)
    pts = rng.normal(size=(4 * len(mons) + 8, 3))
    A = np.stack([pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c for (a, b, c) in mons], axis=1)
    rhs = solid_harmonic(l, m, pts[:, 0], pts[:, 1], pts[:, 2])
    coef, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    resid = np.max(np.abs(A @ coef - rhs))
    if resid > 1e-12 * max(1.0, np.max(np.abs(rhs))):
        raise AssertionError(f"S_{l}{m} is not a degree-{l} polynomial (resid {resid})")
    out = [(e, float(cf)) for e, cf in zip(mons, coef)]
    _POLY_CACHE[key] = out
    return out


def solid_harmonic_grad(l, m, x, y, z):
    """Gradient of S_lm, shape (3,) + x.shape, from its monomial expansion."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    g = np.zeros((3,) + x.shape)
    for (a, b, c), cf in solid_harmonic_poly(l, m):
        if a > 0:
            g[0] += cf * a * x ** (a - 1) * y ** b * z ** c
        if b > 0:
            g[1] += cf * b * x ** a * y ** (b - 1) * z ** c
        if c > 0:
            g[2] += cf * c * x ** a * y ** b * z ** (c - 1)
    return g
