"""Pins for oracle.harmonics and oracle.orbitals (CPU).

What fixes them from outside the oracle:
* the textbook table of real spherical harmonics (p, d, f), typed here from
  the standard definitions, and their quadrature orthonormality;
* solid harmonics are homogeneous harmonic polynomials (Laplacian zero);
* the number of integer points in a ball, by brute-force counting;
* reflection symmetry: an atom on a grid point of a cubic grid gives exactly
  orthonormal grid-normalized orbitals;
* the bounding-box sphere enumeration equals the brute-force test of every
  point of every image.
"""

import itertools

import numpy as np
import pytest

from oracle import harmonics as H
from oracle.orbitals import Site, System, build_sphere, sphere_points, radial_angular, radial_angular_grad

PI = np.pi
TABLE = {
    (1, -1): lambda x, y, z: np.sqrt(3 / (4 * PI)) * y,
    (1, 0): lambda x, y, z: np.sqrt(3 / (4 * PI)) * z,
    (1, 1): lambda x, y, z: np.sqrt(3 / (4 * PI)) * x,
    (2, -2): lambda x, y, z: np.sqrt(15 / (4 * PI)) * x * y,
    (2, -1): lambda x, y, z: np.sqrt(15 / (4 * PI)) * y * z,
    (2, 0): lambda x, y, z: np.sqrt(5 / (16 * PI)) * (3 * z * z - (x * x + y * y + z * z)),
    (2, 1): lambda x, y, z: np.sqrt(15 / (4 * PI)) * x * z,
    (2, 2): lambda x, y, z: np.sqrt(15 / (16 * PI)) * (x * x - y * y),
    (3, -3): lambda x, y, z: np.sqrt(35 / (32 * PI)) * y * (3 * x * x - y * y),
    (3, -2): lambda x, y, z: np.sqrt(105 / (4 * PI)) * x * y * z,
    (3, -1): lambda x, y, z: np.sqrt(21 / (32 * PI)) * y * (5 * z * z - (x * x + y * y + z * z)),
    (3, 0): lambda x, y, z: np.sqrt(7 / (16 * PI)) * z * (5 * z * z - 3 * (x * x + y * y + z * z)),
    (3, 1): lambda x, y, z: np.sqrt(21 / (32 * PI)) * x * (5 * z * z - (x * x + y * y + z * z)),
    (3, 2): lambda x, y, z: np.sqrt(105 / (16 * PI)) * z * (x * x - y * y),
    (3, 3): lambda x, y, z: np.sqrt(35 / (32 * PI)) * x * (x * x - 3 * y * y),
}


def test_real_harmonics_match_textbook_table():
    rng = np.random.default_rng(0)
    p = rng.normal(size=(200, 3))
    for (l, m), fn in TABLE.items():
        got = H.solid_harmonic(l, m, p[:, 0], p[:, 1], p[:, 2])
        np.testing.assert_allclose(got, fn(p[:, 0], p[:, 1], p[:, 2]), rtol=1e-12, atol=1e-12)
    assert np.allclose(H.solid_harmonic(0, 0, p[:, 0], p[:, 1], p[:, 2]), 1 / np.sqrt(4 * PI))


def test_real_harmonics_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(24)
    ph = 2 * PI * np.arange(48) / 48
    CT, PH = np.meshgrid(xg, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    x, y, z = ST * np.cos(PH), ST * np.sin(PH), CT
    W = wg[:, None] * (2 * PI / 48)
    keys = [(l, m) for l in range(4) for m in range(-l, l + 1)]
    Y = [H.real_ylm(l, m, x, y, z) for l, m in keys]
    S = np.array([[np.sum(W * a * b) for b in Y] for a in Y])
    np.testing.assert_allclose(S, np.eye(len(keys)), atol=1e-13)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_solid_harmonics_are_harmonic_and_gradient_consistent(l):
    rng = np.random.default_rng(l)
    p = rng.normal(size=(50, 3))
    eps = 1e-4
    for m in range(-l, l + 1):
        f = lambda q: H.solid_harmonic(l, m, q[:, 0], q[:, 1], q[:, 2])
        lap = np.zeros(len(p))
        g_fd = np.zeros((3, len(p)))
        for ax in range(3):
            e = np.zeros(3)
            e[ax] = eps
            lap += (f(p + e) - 2 * f(p) + f(p - e)) / eps ** 2
            g_fd[ax] = (f(p + e) - f(p - e)) / (2 * eps)
        assert np.max(np.abs(lap)) < 1e-5
        g = H.solid_harmonic_grad(l, m, p[:, 0], p[:, 1], p[:, 2])
        np.testing.assert_allclose(g, g_fd, atol=1e-7)
        # homogeneity of degree l
        np.testing.assert_allclose(f(2.0 * p), 2.0 ** l * f(p), rtol=1e-12, atol=1e-12)


def test_orbital_gradient_matches_finite_difference():
    site = Site(R=np.zeros(3), l=2, zeta=1.7, rc=5.0)
    rng = np.random.default_rng(3)
    d = rng.normal(size=(40, 3))
    eps = 1e-5
    g = radial_angular_grad(site, d)
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = eps
        fd = (radial_angular(site, d + e) - radial_angular(site, d - e)) / (2 * eps)
        np.testing.assert_allclose(g[:, ax, :], fd, atol=1e-8)


def _ball_count(radius_in_h):
    r2 = radius_in_h * radius_in_h
    n = int(radius_in_h)
    return sum(1 for i, j, k in itertools.product(range(-n, n + 1), repeat=3) if i * i + j * j + k * k <= r2)


def test_sphere_point_count_and_ties_on_grid_centre():
    # one d site at (5,5,5) of a 10 bohr cube with 40^3 points, r_c = 16 h
    sys_ = System(cell=[10, 10, 10], ngrid=[40, 40, 40], sites=[Site(R=[5, 5, 5], l=2, zeta=2.0, rc=4.0)])
    g, n, d = sphere_points(sys_, sys_.sites[0])
    assert g.size == _ball_count(16) == 17077
    r = np.sqrt((d * d).sum(1))
    assert np.sum(np.isclose(r, 4.0, rtol=0, atol=1e-12)) == 6     # 16^2 has 6 representations
    assert np.all(n == 0)


@pytest.mark.parametrize("cell,ngrid,R,rc", [
    ([6.0, 6.0, 6.0], [12, 12, 12], [0.1, 5.7, 3.0], 3.4),     # wraps on every axis, self-overlap
    ([4.0, 5.0, 7.0], [8, 10, 14], [0.0, 0.0, 0.0], 2.6),      # atom on a corner
    ([5.0, 5.0, 5.0], [10, 10, 10], [2.3, 1.1, 4.9], 2.0),
])
def test_sphere_bbox_equals_bruteforce(cell, ngrid, R, rc):
    sys_ = System(cell=cell, ngrid=ngrid, sites=[Site(R=R, l=1, zeta=1.0, rc=rc)])
    a = sphere_points(sys_, sys_.sites[0], brute=False)
    b = sphere_points(sys_, sys_.sites[0], brute=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert len(np.unique(a[0])) < a[0].size or rc < min(cell) / 2


def test_grid_orthonormality_symmetric_centre_exact():
    sys_ = System(cell=[10, 10, 10], ngrid=[40, 40, 40], sites=[Site(R=[5, 5, 5], l=2, zeta=2.0, rc=4.0)])
    sp = build_sphere(sys_, sys_.sites[0])
    S = sys_.dV * sp.phi @ sp.phi.T
    assert np.max(np.abs(S - np.eye(5))) < 1e-14
    # an off-grid centre is normalized but only approximately orthogonal
    sys2 = System(cell=[10, 10, 10], ngrid=[40, 40, 40], sites=[Site(R=[5.07, 4.96, 5.11], l=2, zeta=2.0, rc=4.0)])
    sp2 = build_sphere(sys2, sys2.sites[0])
    S2 = sys2.dV * sp2.phi @ sp2.phi.T
    assert np.max(np.abs(np.diag(S2) - 1)) < 1e-14
    assert 1e-9 < np.max(np.abs(S2 - np.eye(5))) < 1e-3
