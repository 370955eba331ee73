"""Pins for oracle.stencil: forces through <phi|grad psi> (Sec. IV).

* Plane waves: the 4th-order central difference of exp(i q.r) on the grid is
  i s(q_i h_i)/h_i times the wave, s(x) = (4/3) sin x - (1/6) sin 2x, at any
  Bloch vector k (not a multiple of the reciprocal lattice), so the stencil
  weights, the 1/h scaling and the phase of neighbours that leave the cell
  are all fixed by a closed form.
* Summation by parts: D is anti-Hermitian on Bloch functions of one k, so
  <phi|D psi> over the sphere points equals -<D Phi_k|psi> over the whole
  cell, with Phi_k the Bloch orbital (spheres that reach past half the cell,
  several images per grid point, collinear and spinor layouts).
* Continuum limit: for smooth states (a few plane waves) and orbitals that
  have decayed at r_c, the force converges to the orbital-derivative force of
  forces.py as h -> 0 (a sign or orientation error gives -F).
* Egg-box: under a rigid sub-grid translation of sites and states the exact
  force is constant; the state-gradient form varies less than the
  orbital-gradient form (the reason Sec. IV gives for it).
"""

import numpy as np
import pytest

from oracle import forces as FO
from oracle import occupations as occ
from oracle import potential as POT
from oracle import projection as P
from oracle import stencil as SG
from oracle.orbitals import Site, System, bloch_orbitals
from tests.helpers import normwise


def _grid_r(sys_, shift=None):
    h = np.asarray(sys_.cell) / np.asarray(sys_.ngrid)
    ix, iy, iz = np.meshgrid(*[np.arange(n) for n in sys_.ngrid], indexing="ij")
    r = np.stack([ix.ravel() * h[0], iy.ravel() * h[1], iz.ravel() * h[2]], axis=1)
    return r if shift is None else r - np.asarray(shift)[None, :]


def _kvec(sys_, ik):
    return 2 * np.pi * np.asarray(sys_.kpts[ik]) / np.asarray(sys_.cell)


def test_plane_wave_symbol():
    sys_ = System(cell=[5.0, 5.5, 6.0], ngrid=[10, 11, 12], sites=[],
                  kpts=np.array([[0.23, -0.31, 0.4], [0.0, 0.45, -0.17]]), kweights=np.full(2, 0.5),
                  spin="collinear")
    r = _grid_r(sys_)
    h = sys_.h
    ms = [np.array([1, -2, 3]), np.array([0, 1, -1]), np.array([-3, 0, 2])]
    psi = np.zeros((sys_.nq, sys_.G, len(ms)), complex)
    qs = np.zeros((sys_.nq, len(ms), 3))
    for q in range(sys_.nq):
        for s, m in enumerate(ms):
            qv = _kvec(sys_, q // sys_.nspin) + 2 * np.pi * m / sys_.cell
            psi[q, :, s] = np.exp(1j * (r @ qv))
            qs[q, s] = qv
    D = SG.fd_gradient(sys_, psi)
    for i in range(3):
        x = qs[..., i] * h[i]
        sym = 1j * ((4.0 / 3.0) * np.sin(x) - (1.0 / 6.0) * np.sin(2 * x)) / h[i]       # (nq, S)
        assert normwise(D[i], psi * sym[:, None, :]) < 1e-13
    # the stencil is 4th order: relative error ~ x^4 / 30 for a long wave
    x = 0.05
    assert abs(((4.0 / 3.0) * np.sin(x) - (1.0 / 6.0) * np.sin(2 * x)) / x - 1.0 + x ** 4 / 30.0) < 1e-9


def _system(spin, cell=(6.0, 6.5, 7.0), ngrid=(12, 13, 14)):
    kpts = ((0.25, -0.25, 0.5), (0.0, 0.25, 0.0))
    return System(cell=list(cell), ngrid=list(ngrid),
                  sites=[Site(R=[0.3, 6.2, 3.3], l=2, zeta=1.6, rc=3.4, species=0),
                         Site(R=[3.1, 3.0, 0.5], l=1, zeta=1.3, rc=2.8, species=1)],
                  kpts=np.array(kpts), kweights=np.full(2, 0.5), spin=spin)


def _random_states(sys_, S, seed):
    rng = np.random.default_rng(seed)
    nsets = sys_.nk if sys_.spin == "spinor" else sys_.nq
    shape = (nsets, sys_.G, S, 2) if sys_.spin == "spinor" else (nsets, sys_.G, S)
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * np.sqrt(1.0 / (sys_.G * sys_.dV))


@pytest.mark.parametrize("spin", ["collinear", "spinor"])
def test_summation_by_parts(spin):
    sys_ = _system(spin)
    sps = P.all_spheres(sys_)
    psi = _random_states(sys_, 3, 4)
    e = SG.state_gradient_projections(sys_, psi, sps)
    off = P.orbital_offsets(sys_)
    for ik in range(sys_.nk):
        one_k = System(cell=list(sys_.cell), ngrid=list(sys_.ngrid), sites=sys_.sites,
                       kpts=sys_.kpts[ik:ik + 1], kweights=np.ones(1), spin="unpolarized")
        qs = [ik] if spin == "spinor" else [ik * 2, ik * 2 + 1]
        for I, (site, sp) in enumerate(zip(sys_.sites, sps)):
            Phi = bloch_orbitals(sys_, site, sys_.kpts[ik], sp)               # (L, G)
            DPhi = SG.fd_gradient(one_k, Phi.T[None])[:, 0]                   # (3, G, L)
            for q in qs:
                for i in range(3):
                    ref = -sys_.dV * (np.conj(DPhi[i]).T @ psi[q].reshape(sys_.G, -1))
                    got = e[q, off[I]:off[I + 1], i].reshape(site.L, -1)
                    assert normwise(got, ref) < 1e-13


def _smooth_states(sys_, S, seed, shift=None, gmax=1):
    """sum over |m_i| <= gmax of a_m exp(i (k + G_m).(r - shift)): smooth
    Bloch states whose rigid translation is known exactly."""
    rng = np.random.default_rng(seed)
    r = _grid_r(sys_, shift)
    psi = np.zeros((sys_.nq, sys_.G, S), complex)
    for q in range(sys_.nq):
        k = _kvec(sys_, q // sys_.nspin)
        for m in np.ndindex(*(2 * gmax + 1,) * 3):
            G = 2 * np.pi * (np.array(m) - gmax) / np.asarray(sys_.cell)
            a = rng.normal(size=S) + 1j * rng.normal(size=S)
            psi[q] += np.exp(1j * (r @ (k + G)))[:, None] * a[None, :]
    return psi / np.sqrt(sys_.G * sys_.dV)


def _both_forces(N, zeta=(2.5, 3.0), rc=(7.0, 6.0), shift=np.zeros(3)):
    R0 = np.array([[1.1, 2.3, 3.05], [4.4, 5.2, 0.7]])
    sys_ = System(cell=[7.2] * 3, ngrid=[N] * 3,
                  sites=[Site(R=R0[0] + shift, l=1, zeta=zeta[0], rc=rc[0]),
                         Site(R=R0[1] + shift, l=2, zeta=zeta[1], rc=rc[1], species=1)],
                  kpts=np.array([[0.1, -0.2, 0.3]]), kweights=np.ones(1), spin="collinear")
    sps = P.all_spheres(sys_)
    psi = _smooth_states(sys_, 3, 1, shift)
    f = np.random.default_rng(2).uniform(0.0, 1.0, size=(sys_.nq, 3))
    c = P.project_sphere(sys_, psi, sps)
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, u, nn) for u, nn in zip((0.35, 0.2), n)]
    Fa = FO.forces_analytic(sys_, c, FO.gradient_projections(sys_, psi, sps), V, f)
    Fs = SG.forces_state_gradient(sys_, c, SG.state_gradient_projections(sys_, psi, sps), V, f)
    return Fa, Fs


def test_continuum_limit_matches_orbital_derivative_form():
    diffs = []
    for N in (24, 48):
        Fa, Fs = _both_forces(N)
        assert np.abs(Fa).max() > 0.1
        diffs.append(np.abs(Fs - Fa).max() / np.abs(Fa).max())
    assert diffs[0] < 5e-3
    assert diffs[1] < 3e-4
    assert diffs[1] < diffs[0] / 8


def test_state_gradient_form_has_smaller_egg_box():
    N = 20
    h = 7.2 / N
    Fa, Fs = [], []
    for t in np.linspace(0.0, 1.0, 7)[:-1]:
        a, s = _both_forces(N, zeta=(2.5, 2.5), rc=(7.0, 6.5), shift=np.array([t * h, 0.37 * t * h, 0.0]))
        Fa.append(a)
        Fs.append(s)
    spread_a = np.ptp(np.array(Fa), axis=0).max()
    spread_s = np.ptp(np.array(Fs), axis=0).max()
    assert spread_s < 0.5 * spread_a
