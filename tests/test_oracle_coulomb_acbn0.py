"""Pins for oracle.coulomb and oracle.acbn0 (CPU).

* G(0): the cell average of 1/r against the closed-form potential of a
  uniform cuboid at its centre (asinh/atan expression, typed here), and its
  1/h scaling.
* Self-energy of a normalized Gaussian, 1/(sigma sqrt(pi)), reached at O(h^2)
  (Richardson extrapolation of two spacings).
* The zero-padded FFT convolution equals the O(N^2) double sum on a small
  sphere (the padding makes the circular convolution linear).
* Tensor symmetries, positive definiteness of the pair matrix, and the
  continuum sum rule sum_{mm'} (mm|m'm') = L^2 F^0.
* Slater integrals: 1s F^0 = 5 zeta / 8 (helium textbook value) and the d-shell
  F^k from exact symbolic integration (sympy).
* Full shell (P-bar = n = 1, both spins): U-bar = 2L F^0 / (2L - 1) and
  J-bar = (2l+1)^2 sum_k F^k (l k l; 0 0 0)^2 / (L (L - 1)) with Wigner 3j
  symbols from sympy, for the continuum tensor.
* The grid tensor approaches the continuum tensor at O(h^2).
* One electron in one orbital: both denominators vanish -> status 1.
* Spinors: single-component spinors reproduce the collinear U-bar, J-bar
  exactly; a global SU(2) rotation leaves the spinor U-bar, J-bar unchanged.
"""

import numpy as np
import pytest

from oracle import acbn0, coulomb
from oracle.orbitals import Site, System, build_sphere


def _cuboid_closed_form(a, b, c):
    r = np.sqrt(a * a + b * b + c * c)
    return (a * b * np.arcsinh(c / np.hypot(a, b)) + b * c * np.arcsinh(a / np.hypot(b, c))
            + c * a * np.arcsinh(b / np.hypot(c, a))
            - 0.5 * a * a * np.arctan(b * c / (a * r)) - 0.5 * b * b * np.arctan(c * a / (b * r))
            - 0.5 * c * c * np.arctan(a * b / (c * r)))


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.25, 0.25, 0.25), (0.24, 0.3, 0.41)])
def test_g0_matches_cuboid_closed_form(h):
    ref = 8 * _cuboid_closed_form(h[0] / 2, h[1] / 2, h[2] / 2) / np.prod(h)
    assert abs(coulomb.g0_box_average(h) - ref) < 1e-12 * ref
    if h[0] == h[1] == h[2]:
        assert abs(coulomb.g0_box_average(h) - 2.380077363979553 / h[0]) < 1e-12 / h[0]


def _gauss_self_energy(h, sigma=1.0, half=6.0):
    n = int(round(2 * half / h)) + 1
    x = (np.arange(n) - (n - 1) / 2) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    rho = (2 * np.pi * sigma ** 2) ** -1.5 * np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * sigma ** 2))
    hh = (h, h, h)
    v = coulomb.hockney_potential(rho[..., None], hh, coulomb.g0_box_average(hh))[..., 0]
    return h ** 3 * np.sum(rho * v)


def test_gaussian_self_energy_second_order():
    exact = 1.0 / np.sqrt(np.pi)
    e1 = _gauss_self_energy(0.25)
    e2 = _gauss_self_energy(0.125)
    r1 = abs(e1 - exact) / exact
    r2 = abs(e2 - exact) / exact
    assert 3.0 < r1 / r2 < 5.0            # O(h^2)
    rich = (4 * e2 - e1) / 3
    assert abs(rich - exact) / exact < 5e-6
    assert r2 < 5e-4


def test_fft_equals_direct_double_sum():
    sys_ = System(cell=[5, 5, 5], ngrid=[10, 10, 10], sites=[Site(R=[0.1, 4.8, 2.6], l=2, zeta=1.8, rc=2.2)])
    sp = build_sphere(sys_, sys_.sites[0])
    Tf = coulomb.coulomb_tensor(sys_, sys_.sites[0], sp, method="fft")
    Td = coulomb.coulomb_tensor(sys_, sys_.sites[0], sp, method="direct")
    assert np.max(np.abs(Tf - Td)) < 1e-13 * np.max(np.abs(Td))


@pytest.fixture(scope="module")
def d_shell_tensors():
    sys_ = System(cell=[10, 10, 10], ngrid=[40, 40, 40], sites=[Site(R=[5, 5, 5], l=2, zeta=2.0, rc=4.0)])
    sp = build_sphere(sys_, sys_.sites[0])
    Tg = coulomb.coulomb_tensor(sys_, sys_.sites[0], sp)
    Tc = coulomb.continuum_tensor(2, 2.0, 4.0)
    return Tg, Tc


def test_tensor_symmetries_and_definiteness(d_shell_tensors):
    for T in d_shell_tensors:
        L = T.shape[0]
        np.testing.assert_allclose(T, T.transpose(1, 0, 2, 3), atol=1e-14)
        np.testing.assert_allclose(T, T.transpose(2, 3, 0, 1), atol=1e-14)
        ev = np.linalg.eigvalsh(T.reshape(L * L, L * L))
        assert ev.min() > -1e-13
        assert ev.max() > 0.5


def test_continuum_sum_rule(d_shell_tensors):
    _, Tc = d_shell_tensors
    F0 = coulomb.slater_Fk(2, 2.0, 4.0, 0)
    assert abs(np.einsum("aacc->", Tc) - 25 * F0) < 1e-12


def test_slater_integrals_closed_forms():
    zeta = 1.7
    assert abs(coulomb.slater_Fk(0, zeta, 40.0, 0) - 5 * zeta / 8) < 1e-11
    sympy = pytest.importorskip("sympy")
    r1, r2, z = sympy.symbols("r1 r2 z", positive=True)
    l = 2
    P = lambda r: r ** (2 * l + 2) * sympy.exp(-2 * z * r)
    norm = sympy.integrate(P(r1), (r1, 0, sympy.oo))
    for k in (0, 2, 4):
        inner = sympy.integrate(P(r2) * r2 ** k, (r2, 0, r1))
        Fk = 2 * sympy.integrate(P(r1) * r1 ** (-(k + 1)) * inner, (r1, 0, sympy.oo)) / norm ** 2
        exact = float(sympy.nsimplify(sympy.simplify(Fk)).subs(z, zeta))
        assert abs(coulomb.slater_Fk(2, zeta, 40.0, k) - exact) < 1e-11 * exact
    assert abs(float(sympy.Rational(793, 3072)) * zeta - coulomb.slater_Fk(2, zeta, 40.0, 0)) < 1e-11


def test_full_shell_closed_forms_continuum(d_shell_tensors):
    from sympy.physics.wigner import wigner_3j
    _, Tc = d_shell_tensors
    l, L = 2, 5
    I = np.stack([np.eye(L), np.eye(L)]).astype(np.complex128)
    U, J, st, im = acbn0.uj_collinear(I, I, Tc)
    F = [coulomb.slater_Fk(l, 2.0, 4.0, k) for k in range(0, 2 * l + 1)]
    assert st == 0 and im < 1e-14
    assert abs(U - 2 * L * F[0] / (2 * L - 1)) < 1e-12
    s = sum(F[k] * float(wigner_3j(l, k, l, 0, 0, 0)) ** 2 for k in range(0, 2 * l + 1))
    assert abs(J - (2 * l + 1) ** 2 * s / (L * (L - 1))) < 1e-12


def test_grid_tensor_converges_to_continuum_second_order():
    errs = []
    for n in (20, 40):
        sys_ = System(cell=[8, 8, 8], ngrid=[n, n, n], sites=[Site(R=[4, 4, 4], l=1, zeta=1.5, rc=3.0)])
        sp = build_sphere(sys_, sys_.sites[0])
        Tg = coulomb.coulomb_tensor(sys_, sys_.sites[0], sp)
        Tc = coulomb.continuum_tensor(1, 1.5, 3.0)
        errs.append(np.max(np.abs(Tg - Tc)) / np.max(np.abs(Tc)))
    assert errs[1] < 1e-2
    assert 2.5 < errs[0] / errs[1] < 6.0


def test_degenerate_single_electron():
    T = np.random.default_rng(0).normal(size=(5, 5, 5, 5))
    n = np.zeros((2, 5, 5), dtype=np.complex128)
    n[0, 2, 2] = 1.0
    U, J, st, _ = acbn0.uj_collinear(n, n, T)
    assert st == 1 and U == 0.0 and J == 0.0


def _random_density(L, rng, scale=0.6):
    A = rng.normal(size=(L, L)) + 1j * rng.normal(size=(L, L))
    H = A @ A.conj().T
    return scale * H / np.linalg.eigvalsh(H).max()


def test_spinor_uj_reduces_and_is_su2_invariant(d_shell_tensors):
    Tg, _ = d_shell_tensors
    rng = np.random.default_rng(4)
    L = 5
    nu, nd = _random_density(L, rng), _random_density(L, rng)
    pu, pd = 0.5 * nu, 0.3 * nd
    Uc, Jc, _, _ = acbn0.uj_collinear(np.stack([nu, nd]), np.stack([pu, pd]), Tg)
    z = np.zeros((L, L))
    ns = np.array([[nu, z], [z, nd]])
    ps = np.array([[pu, z], [z, pd]])
    Us, Js, _, im = acbn0.uj_spinor(ns, ps, Tg)
    assert abs(Us - Uc) < 1e-13 and abs(Js - Jc) < 1e-13
    # global SU(2) rotation: N -> (W x 1) N (W x 1)^dagger
    a, b = rng.normal(size=2) + 1j * rng.normal(size=2)
    W = np.array([[a, -np.conj(b)], [b, np.conj(a)]]) / np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    def rot(M):
        out = np.zeros_like(M, dtype=np.complex128)
        for s in range(2):
            for t in range(2):
                for u in range(2):
                    for v in range(2):
                        out[s, t] += np.conj(W[s, u]) * M[u, v] * W[t, v]
        return out
    Ur, Jr, _, _ = acbn0.uj_spinor(rot(ns), rot(ps), Tg)
    assert abs(Ur - Us) < 1e-12 and abs(Jr - Js) < 1e-12
