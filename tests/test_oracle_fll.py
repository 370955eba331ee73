"""Pins for oracle.fll: the noncollinear HF energy and the FLL double
counting with magnetization (App. A).

* App. A's own reduction: for occupations diagonal in m (any Hermitian 2x2
  spin block per m), E_ee - E_DC equals the rotationally invariant E_U of
  potential.energy at U_eff = U - J (spinor, collinear and unpolarized
  storage).  A dropped or mis-signed term in either formula fails it.
* One electron in a spin-coherent state along (theta, phi), built through
  the occupation pipeline: N = 1 and m the unit vector of that direction
  (fixes the sign convention of m_y).
* A global SU(2) rotation of every spinor rotates m by the matching SO(3)
  rotation (Rodrigues' formula) and leaves N and E_DC unchanged.
* A full shell: N = 2L, m = 0, E_DC = U L(2L-1) - J L(L-1), E_ee = E_DC.
"""

import numpy as np
import pytest

from oracle import fll as FL
from oracle import occupations as occ
from oracle import potential as POT
from oracle.orbitals import Site, System

U, J = 0.31, 0.07


def _sys(spin, l=2):
    return System(cell=[6.0, 6.0, 6.0], ngrid=[8, 8, 8], sites=[Site(R=[0.0, 0.0, 0.0], l=l, zeta=1.5, rc=2.0)],
                  kpts=np.zeros((1, 3)), kweights=np.ones(1), spin=spin)


def _psd_block(rng):
    X = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    H = X @ X.conj().T
    return H / (1.1 * np.linalg.eigvalsh(H).max())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hf_minus_double_counting_is_dudarev_spinor(seed):
    rng = np.random.default_rng(seed)
    sys_ = _sys("spinor")
    L = 5
    n = np.zeros((2, 2, L, L), dtype=np.complex128)
    for a in range(L):
        H = _psd_block(rng)
        for s in range(2):
            for t in range(2):
                n[s, t, a, a] = H[s, t]
    N, m = FL.moments(sys_, n)
    lhs = FL.hf_energy(sys_, n, U, J) - FL.double_counting(N, m, U, J)
    assert abs(lhs - POT.energy(sys_, U - J, n)) < 1e-14
    assert np.linalg.norm(m) > 1e-2


@pytest.mark.parametrize("spin", ["collinear", "unpolarized"])
def test_hf_minus_double_counting_is_dudarev_collinear(spin):
    rng = np.random.default_rng(3)
    sys_ = _sys(spin)
    ns = 2 if spin == "collinear" else 1
    n = np.array([np.diag(rng.uniform(0.0, 1.0, size=5)) for _ in range(ns)]).astype(np.complex128)
    N, m = FL.moments(sys_, n)
    lhs = FL.hf_energy(sys_, n, U, J) - FL.double_counting(N, m, U, J)
    assert abs(lhs - POT.energy(sys_, U - J, n)) < 1e-14
    if spin == "unpolarized":
        assert np.all(m == 0.0)
        assert abs(N - 2 * np.trace(n[0]).real) < 1e-15


def _spinor(theta, phi):
    return np.array([np.cos(theta / 2), np.exp(1j * phi) * np.sin(theta / 2)])


@pytest.mark.parametrize("theta,phi", [(0.0, 0.0), (np.pi, 0.0), (np.pi / 2, 0.0), (np.pi / 2, np.pi / 2),
                                       (1.1, -2.3)])
def test_spin_coherent_state(theta, phi):
    sys_ = _sys("spinor", l=1)
    c = np.zeros((1, 3, 1, 2), dtype=np.complex128)
    c[0, 1, 0] = _spinor(theta, phi) * np.exp(0.7j)              # any global phase
    n, _, _ = occ.occupations(sys_, c, np.ones((1, 1)), with_pbar=False)
    N, m = FL.moments(sys_, n[0])
    assert abs(N - 1.0) < 1e-14
    ref = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    assert np.max(np.abs(m - ref)) < 1e-14


def test_global_spin_rotation():
    rng = np.random.default_rng(4)
    sys_ = _sys("spinor")
    S = 6
    c = rng.normal(size=(1, 5, S, 2)) + 1j * rng.normal(size=(1, 5, S, 2))
    f = rng.uniform(0.0, 1.0, size=(1, S))
    axis = np.array([0.3, -0.5, 0.8])
    axis /= np.linalg.norm(axis)
    ang = 1.234
    sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    U2 = np.cos(ang / 2) * np.eye(2) - 1j * np.sin(ang / 2) * sum(a * s for a, s in zip(axis, sig))
    c_rot = np.einsum("st,kjnt->kjns", U2, c)
    n0, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    n1, _, _ = occ.occupations(sys_, c_rot, f, with_pbar=False)
    N0, m0 = FL.moments(sys_, n0[0])
    N1, m1 = FL.moments(sys_, n1[0])
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
    assert abs(N1 - N0) < 1e-12 * N0
    assert np.max(np.abs(m1 - R @ m0)) < 1e-12 * np.linalg.norm(m0)
    assert abs(FL.double_counting(N1, m1, U, J) - FL.double_counting(N0, m0, U, J)) < 1e-12


def test_full_shell():
    sys_ = _sys("spinor")
    L = 5
    n = np.zeros((2, 2, L, L), dtype=np.complex128)
    n[0, 0] = n[1, 1] = np.eye(L)
    N, m = FL.moments(sys_, n)
    assert N == 2 * L and np.all(m == 0.0)
    edc = FL.double_counting(N, m, U, J)
    assert abs(edc - (U * L * (2 * L - 1) - J * L * (L - 1))) < 1e-14
    assert abs(FL.hf_energy(sys_, n, U, J) - edc) < 1e-13
