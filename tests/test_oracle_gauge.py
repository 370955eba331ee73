"""Pins for oracle.gauge: the velocity-gauge operator and current (Sec. V).

* A = 0 reduces the gauge projection and apply to the plain sphere forms.
* Gauge covariance, for any A (not only lattice-commensurate ones): the
  gauge projection of psi at crystal momentum k equals the plain projection
  (``project_sphere``) of the modulated state exp(i A.r_g) psi, a Bloch state
  at k + A; the gauge apply equals exp(-i A.r_g) times the plain full-grid
  apply at k + A.  The spheres used reach past half the cell, so grid points
  are hit through several lattice images: a phase taken at the folded point
  r_g instead of the unfolded r_p fails this.
* The current equals the derivative of sum w f <psi|V^A|psi> in A with V
  held fixed (central finite differences, per site), collinear and spinor.
* V^A is Hermitian; real Gamma-point states at A = 0 carry no current.
"""

import numpy as np
import pytest

from oracle import gauge as GA
from oracle import occupations as occ
from oracle import potential as POT
from oracle import projection as P
from oracle import step as ST
from oracle.orbitals import Site, System
from tests.helpers import normwise


def _system(spin="collinear", kpts=((0.25, -0.25, 0.5), (0.0, 0.25, 0.0))):
    return System(cell=[6.0, 6.5, 7.0], ngrid=[12, 13, 14],
                  sites=[Site(R=[0.3, 6.2, 3.3], l=2, zeta=1.6, rc=3.4, species=0),
                         Site(R=[3.1, 3.0, 0.5], l=1, zeta=1.3, rc=2.8, species=1)],
                  kpts=np.array(kpts), kweights=np.full(len(kpts), 1.0 / len(kpts)), spin=spin)


def _shifted(sys_, A):
    """The same system at crystal momenta k + A (reduced units per axis)."""
    dk = np.asarray(A) * np.asarray(sys_.cell) / (2 * np.pi)
    return System(cell=list(sys_.cell), ngrid=list(sys_.ngrid), sites=sys_.sites,
                  kpts=np.asarray(sys_.kpts) + dk[None, :], kweights=sys_.kweights, spin=sys_.spin)


def _grid_r(sys_):
    h = np.asarray(sys_.cell) / np.asarray(sys_.ngrid)
    ix, iy, iz = np.meshgrid(*[np.arange(n) for n in sys_.ngrid], indexing="ij")
    return np.stack([ix.ravel() * h[0], iy.ravel() * h[1], iz.ravel() * h[2]], axis=1)


def _states(sys_, S, seed):
    rng = np.random.default_rng(seed)
    nsets = sys_.nk if sys_.spin == "spinor" else sys_.nq
    shape = (nsets, sys_.G, S, 2) if sys_.spin == "spinor" else (nsets, sys_.G, S)
    psi = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return psi * np.sqrt(1.0 / (sys_.G * sys_.dV))


def _potentials(sys_, c, f, ueffs=(0.35, 0.2)):
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    return [POT.potential_matrix(sys_, u, nn) for u, nn in zip(ueffs, n)]


def _occ(sys_, S, seed):
    rng = np.random.default_rng(seed)
    nsets = sys_.nk if sys_.spin == "spinor" else sys_.nq
    return rng.uniform(0.0, 1.0, size=(nsets, S))


A_GENERIC = np.array([0.137, -0.291, 0.083])


@pytest.mark.parametrize("spin", ["collinear", "spinor"])
def test_zero_field_reduces_to_plain_forms(spin):
    sys_ = _system(spin)
    sps = P.all_spheres(sys_)
    psi = _states(sys_, 5, 1)
    f = _occ(sys_, 5, 2)
    c0 = P.project_sphere(sys_, psi, sps)
    cA = GA.project_gauge(sys_, psi, sps, np.zeros(3))
    assert normwise(cA, c0) < 1e-14
    V = _potentials(sys_, c0, f)
    assert normwise(GA.apply_gauge(sys_, c0, V, sps, np.zeros(3)), ST.apply_sphere(sys_, c0, V, sps)) < 1e-14


@pytest.mark.parametrize("spin", ["collinear", "spinor"])
def test_gauge_projection_is_shifted_crystal_momentum(spin):
    sys_ = _system(spin)
    sps = P.all_spheres(sys_)
    psi = _states(sys_, 4, 3)
    mod = np.exp(1j * (_grid_r(sys_) @ A_GENERIC))
    psi_mod = psi * (mod[None, :, None, None] if spin == "spinor" else mod[None, :, None])
    sh = _shifted(sys_, A_GENERIC)
    cA = GA.project_gauge(sys_, psi, sps, A_GENERIC)
    ref = P.project_sphere(sh, psi_mod, P.all_spheres(sh))
    assert normwise(cA, ref) < 1e-13
    # and it is not the folded-point phase
    folded = P.project_sphere(sys_, psi_mod, sps)
    assert normwise(folded, ref) > 1e-3


@pytest.mark.parametrize("spin", ["collinear", "spinor"])
def test_gauge_apply_is_shifted_crystal_momentum(spin):
    sys_ = _system(spin)
    sps = P.all_spheres(sys_)
    psi = _states(sys_, 4, 5)
    f = _occ(sys_, 4, 6)
    cA = GA.project_gauge(sys_, psi, sps, A_GENERIC)
    V = _potentials(sys_, cA, f)
    out = GA.apply_gauge(sys_, cA, V, sps, A_GENERIC)
    sh = _shifted(sys_, A_GENERIC)
    ref = POT.apply_fullgrid(sh, cA, V, P.all_spheres(sh))
    demod = np.exp(-1j * (_grid_r(sys_) @ A_GENERIC))
    ref = ref * (demod[None, :, None, None] if spin == "spinor" else demod[None, :, None])
    assert normwise(out, ref) < 1e-13


def _site_expectation(sys_, c, V, f, I):
    off = P.orbital_offsets(sys_)
    mask = np.zeros(c.shape[1], bool)
    mask[off[I]:off[I + 1]] = True
    cI = np.where(mask[None, :, None, None] if sys_.spin == "spinor" else mask[None, :, None], c, 0.0)
    return GA.expectation(sys_, cI, V, f)


@pytest.mark.parametrize("spin", ["collinear", "unpolarized", "spinor"])
def test_current_is_field_derivative(spin):
    kpts = ((0.0, 0.0, 0.0),) if spin == "unpolarized" else ((0.25, -0.25, 0.5), (0.0, 0.25, 0.0))
    sys_ = _system(spin, kpts)
    sps = P.all_spheres(sys_)
    psi = _states(sys_, 4, 7)
    f = _occ(sys_, 4, 8)
    cA = GA.project_gauge(sys_, psi, sps, A_GENERIC)
    V = _potentials(sys_, cA, f)                                  # held fixed below
    rho = GA.moment_projections(sys_, psi, sps, A_GENERIC)
    J = GA.current(sys_, cA, rho, V, f)
    delta = 1e-5
    fd = np.zeros_like(J)
    for i in range(3):
        e = np.zeros(3)
        e[i] = delta
        cp = GA.project_gauge(sys_, psi, sps, A_GENERIC + e)
        cm = GA.project_gauge(sys_, psi, sps, A_GENERIC - e)
        for I in range(len(sys_.sites)):
            fd[I, i] = (_site_expectation(sys_, cp, V, f, I) - _site_expectation(sys_, cm, V, f, I)) / (2 * delta)
    assert np.max(np.abs(J)) > 1e-4
    assert np.max(np.abs(J - fd)) < 1e-7 * np.max(np.abs(J))


def test_gauge_operator_is_hermitian():
    sys_ = _system("collinear")
    sps = P.all_spheres(sys_)
    psi = _states(sys_, 3, 9)
    chi = _states(sys_, 3, 10)
    f = _occ(sys_, 3, 11)
    V = _potentials(sys_, GA.project_gauge(sys_, psi, sps, A_GENERIC), f)
    Vpsi = GA.apply_gauge(sys_, GA.project_gauge(sys_, psi, sps, A_GENERIC), V, sps, A_GENERIC)
    Vchi = GA.apply_gauge(sys_, GA.project_gauge(sys_, chi, sps, A_GENERIC), V, sps, A_GENERIC)
    lhs = np.einsum("qgs,qgs->qs", np.conj(chi), Vpsi)
    rhs = np.conj(np.einsum("qgs,qgs->qs", np.conj(psi), Vchi))
    assert normwise(lhs, rhs) < 1e-13


def test_real_gamma_states_carry_no_current():
    sys_ = _system("unpolarized", ((0.0, 0.0, 0.0),))
    sps = P.all_spheres(sys_)
    psi = _states(sys_, 4, 12).real.astype(np.complex128)
    f = _occ(sys_, 4, 13)
    c = GA.project_gauge(sys_, psi, sps, np.zeros(3))
    V = _potentials(sys_, c, f)
    J = GA.current(sys_, c, GA.moment_projections(sys_, psi, sps, np.zeros(3)), V, f)
    assert np.max(np.abs(J)) < 1e-14
    # a field breaks it
    cA = GA.project_gauge(sys_, psi, sps, A_GENERIC)
    VA = _potentials(sys_, cA, f)
    JA = GA.current(sys_, cA, GA.moment_projections(sys_, psi, sps, A_GENERIC), VA, f)
    assert np.max(np.abs(JA)) > 1e-6
