"""Pins for oracle.spinorb: spin-dependent orbitals of noncollinear runs
(App. A).

* Without a spin-down exponent (or with zeta_dn = zeta) the projection and
  the apply are the spin-independent spinor forms of projection.py and
  potential.py.
* With zeta_dn != zeta: the sphere forms equal the full-cell definitions
  (spheres past half the cell); a state with only one spin component
  projects like a one-component state onto that component's orbital.
* V_U psi is the derivative of E_U with these projections: central finite
  differences of sum_I E_U along a random direction give
  2 Re sum dV w f <delta|V_U psi>.
"""

import numpy as np
import pytest

from oracle import occupations as occ
from oracle import potential as POT
from oracle import projection as P
from oracle import spinorb as SO
from oracle.orbitals import Site, System
from tests.helpers import normwise


def _system(zdn=(2.3, None)):
    return System(cell=[6.0, 6.5, 7.0], ngrid=[12, 13, 14],
                  sites=[Site(R=[0.3, 6.2, 3.3], l=2, zeta=1.6, rc=3.4, species=0, zeta_dn=zdn[0]),
                         Site(R=[3.1, 3.0, 0.5], l=1, zeta=1.3, rc=2.8, species=1, zeta_dn=zdn[1])],
                  kpts=np.array([[0.25, -0.25, 0.5], [0.0, 0.25, 0.0]]), kweights=np.full(2, 0.5), spin="spinor")


def _states(sys_, S, seed):
    rng = np.random.default_rng(seed)
    shape = (sys_.nk, sys_.G, S, 2)
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * np.sqrt(1.0 / (sys_.G * sys_.dV))


def _V(sys_, c, f, ueffs=(0.35, 0.2)):
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    return [POT.potential_matrix(sys_, u, nn) for u, nn in zip(ueffs, n)], n


@pytest.mark.parametrize("zdn", [(None, None), (1.6, 1.3)])
def test_spin_independent_limit(zdn):
    sys_ = _system(zdn)
    psi = _states(sys_, 3, 1)
    f = np.random.default_rng(2).uniform(0.0, 1.0, size=(sys_.nk, 3))
    c = SO.project_spin(sys_, psi)
    ref = P.project_fullgrid(sys_, psi)
    assert normwise(c, ref) < 1e-13
    V, _ = _V(sys_, c, f)
    assert normwise(SO.apply_spin(sys_, c, V), POT.apply_fullgrid(sys_, c, V)) < 1e-13


def test_sphere_form_equals_definition():
    sys_ = _system()
    psi = _states(sys_, 3, 3)
    f = np.random.default_rng(4).uniform(0.0, 1.0, size=(sys_.nk, 3))
    c = SO.project_spin(sys_, psi)
    assert normwise(SO.project_spin(sys_, psi, form="sphere"), c) < 1e-13
    assert normwise(c, P.project_fullgrid(sys_, psi)) > 1e-3        # the spin-down orbitals differ
    V, _ = _V(sys_, c, f)
    assert normwise(SO.apply_spin(sys_, c, V, form="sphere"), SO.apply_spin(sys_, c, V)) < 1e-13


@pytest.mark.parametrize("sg", [0, 1])
def test_single_component_states(sg):
    sys_ = _system()
    psi = _states(sys_, 3, 5)
    psi[..., 1 - sg] = 0.0
    c = SO.project_spin(sys_, psi)
    assert np.all(c[..., 1 - sg] == 0.0)
    zeta = [s.zeta if sg == 0 or s.zeta_dn is None else s.zeta_dn for s in sys_.sites]
    one = System(cell=sys_.cell, ngrid=sys_.ngrid,
                 sites=[Site(R=s.R, l=s.l, zeta=z, rc=s.rc, species=s.species) for s, z in zip(sys_.sites, zeta)],
                 kpts=sys_.kpts, kweights=sys_.kweights, spin="unpolarized")
    assert normwise(c[..., sg], P.project_sphere(one, psi[..., sg], P.all_spheres(one))) < 1e-13


def _energy(sys_, psi, f, ueffs):
    c = SO.project_spin(sys_, psi, form="sphere")
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    return sum(POT.energy(sys_, u, nn) for u, nn in zip(ueffs, n))


def test_apply_is_energy_derivative():
    sys_ = _system()
    psi = _states(sys_, 3, 6)
    f = np.random.default_rng(7).uniform(0.0, 1.0, size=(sys_.nk, 3))
    ueffs = (0.35, 0.2)
    c = SO.project_spin(sys_, psi, form="sphere")
    V, _ = _V(sys_, c, f, ueffs)
    hpsi = SO.apply_spin(sys_, c, V, form="sphere")
    rng = np.random.default_rng(8)
    delta = rng.normal(size=psi.shape) + 1j * rng.normal(size=psi.shape)
    eps = 1e-5
    fd = (_energy(sys_, psi + eps * delta, f, ueffs) - _energy(sys_, psi - eps * delta, f, ueffs)) / (2 * eps)
    wf = sys_.kweights[:, None] * f
    an = 2.0 * sys_.dV * np.sum(np.conj(delta) * hpsi * wf[:, None, :, None]).real
    assert abs(an) > 1e-6
    assert abs(fd - an) < 1e-7 * abs(an)


def test_forces_are_position_derivative():
    """F from the components' orbital gradients = central FD of E_U in R
    (frozen sphere points and normalization, both components moved)."""
    from oracle import forces as FO
    from oracle.orbitals import build_sphere
    sys_ = _system()
    psi = _states(sys_, 3, 11)
    f = np.random.default_rng(12).uniform(0.0, 1.0, size=(sys_.nk, 3))
    ueffs = (0.35, 0.2)
    comps = SO.component_systems(sys_)
    ref = [[build_sphere(cs, s) for s in cs.sites] for cs in comps]

    def energy(I, i, dR):
        cs_list = []
        for cs, sps in zip(comps, ref):
            sp = list(sps)
            R = cs.sites[I].R.copy()
            R[i] += dR
            sp[I] = build_sphere(cs, cs.sites[I], R_eval=R, norms=sps[I].norms)
            cs_list.append(sp)
        c = np.stack([P.project_sphere(cs, psi[..., sg], sps) for sg, (cs, sps) in enumerate(zip(comps, cs_list))],
                     axis=-1)
        n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
        return sum(POT.energy(sys_, u, nn) for u, nn in zip(ueffs, n))

    c = SO.project_spin(sys_, psi, form="sphere")
    V, _ = _V(sys_, c, f, ueffs)
    F = FO.forces_analytic(sys_, c, SO.gradient_projections_spin(sys_, psi), V, f)
    delta = 1e-4
    for I in range(2):
        for i in range(3):
            fd = -(energy(I, i, delta) - energy(I, i, -delta)) / (2 * delta)
            assert abs(F[I, i] - fd) < 1e-6 * max(1.0, np.abs(F).max()), (I, i)
    assert np.abs(F).max() > 1e-4


def test_current_is_field_derivative():
    """J from the components' position moments = central FD in A of the
    site's sum w f <psi|V^A|psi> with V fixed."""
    from oracle import gauge as GA
    sys_ = _system()
    psi = _states(sys_, 3, 13)
    f = np.random.default_rng(14).uniform(0.0, 1.0, size=(sys_.nk, 3))
    A = np.array([0.137, -0.291, 0.083])
    cA = SO.project_gauge_spin(sys_, psi, A)
    V, _ = _V(sys_, cA, f)
    J = GA.current(sys_, cA, SO.moment_projections_spin(sys_, psi, A), V, f)
    off = P.orbital_offsets(sys_)

    def site_e(c, I):
        mask = np.zeros(c.shape[1], bool)
        mask[off[I]:off[I + 1]] = True
        return GA.expectation(sys_, np.where(mask[None, :, None, None], c, 0.0), V, f)

    delta = 1e-5
    for i in range(3):
        e = np.zeros(3)
        e[i] = delta
        cp, cm = SO.project_gauge_spin(sys_, psi, A + e), SO.project_gauge_spin(sys_, psi, A - e)
        for I in range(2):
            fd = (site_e(cp, I) - site_e(cm, I)) / (2 * delta)
            assert abs(J[I, i] - fd) < 1e-7 * np.abs(J).max(), (I, i)
    assert np.abs(J).max() > 1e-4


def _grid_r(sys_):
    h = np.asarray(sys_.cell) / np.asarray(sys_.ngrid)
    ix, iy, iz = np.meshgrid(*[np.arange(n) for n in sys_.ngrid], indexing="ij")
    return np.stack([ix.ravel() * h[0], iy.ravel() * h[1], iz.ravel() * h[2]], axis=1)


def test_gauge_forms():
    """A = 0 gives the plain spin-dependent forms; for any A the gauge
    projection and apply are the plain ones at k + A of exp(i A.r) psi."""
    sys_ = _system()
    psi = _states(sys_, 3, 15)
    f = np.random.default_rng(16).uniform(0.0, 1.0, size=(sys_.nk, 3))
    c0 = SO.project_spin(sys_, psi, form="sphere")
    V, _ = _V(sys_, c0, f)
    assert normwise(SO.project_gauge_spin(sys_, psi, np.zeros(3)), c0) < 1e-14
    assert normwise(SO.apply_gauge_spin(sys_, c0, V, np.zeros(3)), SO.apply_spin(sys_, c0, V, form="sphere")) < 1e-14
    A = np.array([0.137, -0.291, 0.083])
    dk = A * np.asarray(sys_.cell) / (2 * np.pi)
    sh = System(cell=sys_.cell, ngrid=sys_.ngrid, sites=sys_.sites, kpts=np.asarray(sys_.kpts) + dk[None, :],
                kweights=sys_.kweights, spin="spinor")
    mod = np.exp(1j * (_grid_r(sys_) @ A))[None, :, None, None]
    cA = SO.project_gauge_spin(sys_, psi, A)
    assert normwise(cA, SO.project_spin(sh, psi * mod, form="sphere")) < 1e-13
    VA, _ = _V(sys_, cA, f)
    assert normwise(SO.apply_gauge_spin(sys_, cA, VA, A) * mod, SO.apply_spin(sh, cA, VA, form="sphere")) < 1e-13


def test_state_gradient_projections():
    """Equal exponents give stencil.py's spinor result; a state with only a
    spin-down component projects like a one-component state onto the
    spin-down orbital."""
    from oracle import stencil as SG
    same = _system(zdn=(1.6, 1.3))
    psi = _states(same, 3, 17)
    e = SO.state_gradient_projections_spin(same, psi)
    assert normwise(e, SG.state_gradient_projections(same, psi, P.all_spheres(same))) < 1e-13
    sys_ = _system()
    psi[..., 0] = 0.0
    e = SO.state_gradient_projections_spin(sys_, psi)
    assert np.all(e[..., 0] == 0.0)
    one = System(cell=sys_.cell, ngrid=sys_.ngrid,
                 sites=[Site(R=s.R, l=s.l, zeta=s.zeta_dn if s.zeta_dn is not None else s.zeta, rc=s.rc,
                             species=s.species) for s in sys_.sites],
                 kpts=sys_.kpts, kweights=sys_.kweights, spin="unpolarized")
    ref = SG.state_gradient_projections(one, psi[..., 1], P.all_spheres(one))
    assert normwise(e[..., 1], ref) < 1e-13
