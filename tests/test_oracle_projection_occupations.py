"""Pins for oracle.projection and oracle.occupations (CPU).

* The sphere-gather form equals the full-grid image sum (the definition).
* Phase convention: a Bloch state of a small primitive cell, where the
  sphere wraps, projects to the same value as the same state laid out on a
  3x3x3 supercell at Gamma, where the sphere does not wrap and no phase is
  needed.  A wrong sign of k.T or a wrong image fails this.
* Lattice covariance: moving the atom by a lattice vector T multiplies c by
  exp(i k.T) and leaves n unchanged.
* psi = phi_m (symmetric centre) gives n = e_m e_m^T exactly.
* n is Hermitian, PSD, with eigenvalues in [0, 1] for orthonormal states and
  orbitals, and invariant under unitary mixing of equally occupied states.
* N-bar lies in [0, 1] for non-overlapping same-species spheres (Sec. III);
  N-bar = 1 gives P-bar = n; N-bar = 0 gives P-bar = 0 (Sec. III limits).
* Sharding the states into groups and summing partial n and P-bar (the
  multi-GPU all-reduce design) reproduces the unsharded result.
* Spinors with a single non-zero component reproduce the collinear result
  (App. B: the spinor P-bar reduces to the usual one on the spin diagonal).
"""

import numpy as np
import pytest

from oracle import occupations as occ
from oracle import projection as P
from oracle.orbitals import Site, System, build_sphere
from synth import make_config, make_occupations, make_states
from tests.helpers import normwise, to_system


def _rand_states(sys_, S, seed, cplx=True):
    rng = np.random.default_rng(seed)
    G = sys_.G
    out = []
    for q in range(sys_.nq):
        A = rng.normal(size=(G, S)) + (1j * rng.normal(size=(G, S)) if cplx else 0)
        Q, _ = np.linalg.qr(A)
        out.append(Q / np.sqrt(sys_.dV))
    return np.stack(out)


def test_sphere_form_equals_fullgrid_with_wrap_and_kpoints():
    sys_ = System(cell=[6.0, 6.5, 7.0], ngrid=[12, 13, 14],
                  sites=[Site(R=[0.2, 6.1, 3.3], l=2, zeta=1.5, rc=3.6, species=0),
                         Site(R=[3.0, 3.1, 0.4], l=1, zeta=1.2, rc=2.9, species=1)],
                  kpts=[[0.25, -0.25, 0.5], [0.0, 0.0, 0.0]], kweights=[0.5, 0.5], spin="collinear")
    psi = _rand_states(sys_, 7, 1)
    a = P.project_fullgrid(sys_, psi)
    b = P.project_sphere(sys_, psi)
    assert normwise(b, a) < 1e-13


def test_phase_convention_against_supercell():
    a = 6.0
    n = 12
    k = np.array([1 / 3, -1 / 3, 1 / 3])
    site = dict(R=[0.3137, 5.8219, 2.9071], l=2, zeta=1.4, rc=3.7)   # no grid point near |d| = r_c
    prim = System(cell=[a] * 3, ngrid=[n] * 3, sites=[Site(**site)], kpts=[k], kweights=[1.0])
    sup = System(cell=[3 * a] * 3, ngrid=[3 * n] * 3,
                 sites=[Site(R=np.array(site["R"]) + a, l=2, zeta=1.4, rc=3.7)])
    rng = np.random.default_rng(7)
    u = rng.normal(size=(n, n, n, 3)) + 1j * rng.normal(size=(n, n, n, 3))     # periodic part
    h = a / n
    def bloch_on(N):
        idx = np.arange(N)
        X, Y, Z = np.meshgrid(idx * h, idx * h, idx * h, indexing="ij")
        ph = np.exp(1j * 2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) / a)
        uu = u[np.ix_(idx % n, idx % n, idx % n)]
        return (uu * ph[..., None]).reshape(-1, 3)
    c_prim = P.project_fullgrid(prim, bloch_on(n)[None])
    c_sup = P.project_fullgrid(sup, bloch_on(3 * n)[None])
    sp = build_sphere(sup, sup.sites[0])
    assert np.all(sp.n == 0)                                   # no wrap in the supercell
    assert np.any(build_sphere(prim, prim.sites[0]).n != 0)    # wraps in the primitive cell
    # the supercell centre is shifted by a lattice vector T0 = (a, a, a): factor exp(i k.T0)
    np.testing.assert_allclose(c_sup, c_prim * np.exp(2j * np.pi * k.sum()), rtol=1e-12, atol=1e-13)


def test_lattice_translation_covariance():
    base = dict(l=1, zeta=1.3, rc=3.2)
    k = np.array([0.25, 0.5, -0.25])
    s0 = System(cell=[6, 6, 6], ngrid=[12, 12, 12], sites=[Site(R=[1.0, 2.0, 3.0], **base)], kpts=[k], kweights=[1.0])
    T = np.array([6.0, -12.0, 6.0])
    s1 = System(cell=[6, 6, 6], ngrid=[12, 12, 12], sites=[Site(R=np.array([1.0, 2.0, 3.0]) + T, **base)], kpts=[k], kweights=[1.0])
    psi = _rand_states(s0, 4, 3)
    c0 = P.project_fullgrid(s0, psi)
    c1 = P.project_fullgrid(s1, psi)
    np.testing.assert_allclose(c1, c0 * np.exp(2j * np.pi * (k @ (T / 6.0))), atol=1e-13)
    f = np.ones((1, 4)) * 0.7
    n0 = occ.occupations(s0, c0, f)[0][0]
    n1 = occ.occupations(s1, c1, f)[0][0]
    np.testing.assert_allclose(n1, n0, atol=1e-14)


def test_state_equal_to_orbital_gives_unit_occupation():
    sys_ = System(cell=[10, 10, 10], ngrid=[40, 40, 40], sites=[Site(R=[5, 5, 5], l=2, zeta=2.0, rc=4.0)])
    sp = build_sphere(sys_, sys_.sites[0])
    Phi = P.bloch_matrix(sys_, np.zeros(3), [sp])
    for m in range(5):
        psi = Phi[m].real.copy()[None, :, None]
        c = P.project_fullgrid(sys_, psi, [sp])
        n, pbar, nb = occ.occupations(sys_, c, np.ones((1, 1)))
        e = np.zeros((5, 5))
        e[m, m] = 1.0
        assert np.max(np.abs(n[0][0] - e)) < 1e-14
        assert abs(nb[0, 0, 0] - 1.0) < 1e-14
        assert np.max(np.abs(pbar[0][0] - n[0][0])) < 1e-14


def _small_nonoverlap_system(spin="collinear", kpts=((0.25, 0.25, 0.0), (-0.25, 0.0, 0.5))):
    return System(cell=[12.0, 12.0, 12.0], ngrid=[24, 24, 24],
                  sites=[Site(R=[6.0, 6.0, 6.0], l=2, zeta=2.0, rc=3.0, species=0),
                         Site(R=[0.0, 0.0, 0.0], l=2, zeta=2.0, rc=3.0, species=0),
                         Site(R=[6.0, 0.0, 6.0], l=1, zeta=1.5, rc=2.5, species=1)],
                  kpts=np.array(kpts), kweights=np.full(len(kpts), 1.0 / len(kpts)), spin=spin)


def test_occupation_invariants():
    sys_ = _small_nonoverlap_system()
    S = 9
    psi = _rand_states(sys_, S, 11)
    # make the states strongly localized on the orbitals so the test is not trivial
    sps = P.all_spheres(sys_)
    rng = np.random.default_rng(2)
    for q in range(sys_.nq):
        Phi = P.bloch_matrix(sys_, sys_.kpts[q // 2], sps)
        A = psi[q] * 0.3 + Phi.T @ (rng.normal(size=(Phi.shape[0], S)) + 1j * rng.normal(size=(Phi.shape[0], S)))
        Q, _ = np.linalg.qr(A)
        psi[q] = Q / np.sqrt(sys_.dV)
    f = rng.uniform(0, 1, size=(sys_.nq, S))
    f[:, :3] = 1.0
    c = P.project_fullgrid(sys_, psi, sps)
    n, pbar, nb = occ.occupations(sys_, c, f)
    for I in range(3):
        for ch in range(2):
            m = n[I][ch]
            assert np.max(np.abs(m - m.conj().T)) < 1e-14
            ev = np.linalg.eigvalsh(m)
            assert ev.min() > -1e-13 and ev.max() < 1 + 1e-12
            assert ev.max() > 0.2
    assert nb.min() >= -1e-15 and nb.max() <= 1 + 1e-12 and nb.max() > 0.5
    # unitary mixing of the three states with f = 1 in every set
    U, _ = np.linalg.qr(rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
    psi2 = psi.copy()
    psi2[:, :, :3] = psi[:, :, :3] @ U
    n2 = occ.occupations(sys_, P.project_fullgrid(sys_, psi2, sps), f)[0]
    for I in range(3):
        np.testing.assert_allclose(n2[I], n[I], atol=1e-13)
    # sharding the states in two groups and summing the partial matrices
    h1 = occ.occupations(sys_, c[:, :, :4], f[:, :4])
    h2 = occ.occupations(sys_, c[:, :, 4:], f[:, 4:])
    for I in range(3):
        np.testing.assert_allclose(h1[0][I] + h2[0][I], n[I], atol=1e-14)
        np.testing.assert_allclose(h1[1][I] + h2[1][I], pbar[I], atol=1e-14)


def test_nbar_limits():
    sys_ = _small_nonoverlap_system(kpts=((0.0, 0.0, 0.0),))
    sps = P.all_spheres(sys_)
    Phi = P.bloch_matrix(sys_, np.zeros(3), sps).real
    # states inside the orbital span of species 0: N-bar = 1 and P-bar = n
    Q, _ = np.linalg.qr(Phi[:10].T)
    psi = np.stack([Q / np.sqrt(sys_.dV)] * 2)
    f = np.ones((2, 10))
    c = P.project_fullgrid(sys_, psi, sps)
    n, pbar, nb = occ.occupations(sys_, c, f)
    assert np.max(np.abs(nb[:, 0, :] - 1.0)) < 1e-12
    for I in (0, 1):
        np.testing.assert_allclose(pbar[I], n[I], atol=1e-12)
    # states orthogonal to every orbital: N-bar = 0 and P-bar = 0
    rng = np.random.default_rng(5)
    A = rng.normal(size=(sys_.G, 6))
    Qo, _ = np.linalg.qr(Phi.T)
    A = A - Qo @ (Qo.T @ A)
    A, _ = np.linalg.qr(A)
    psi0 = np.stack([A / np.sqrt(sys_.dV)] * 2)
    c0 = P.project_fullgrid(sys_, psi0, sps)
    n0, p0, nb0 = occ.occupations(sys_, c0, np.ones((2, 6)))
    assert np.max(np.abs(nb0)) < 1e-24
    assert max(np.max(np.abs(x)) for x in p0) < 1e-24


def test_spinor_with_single_components_reduces_to_collinear():
    cfg = make_config("spinor_layers", small=True)
    sys_s = to_system(cfg)
    sys_c = to_system(cfg)
    sys_c.spin = "collinear"
    rng = np.random.default_rng(9)
    S = 6
    coll = _rand_states(sys_c, S, 4)                                   # [k*2 + sigma][G][S]
    spin = np.zeros((sys_s.nk, sys_s.G, 2 * S, 2), dtype=np.complex128)
    f_c = rng.uniform(0, 1, size=(sys_c.nq, S))
    f_s = np.zeros((sys_s.nk, 2 * S))
    for ik in range(sys_s.nk):
        for sg in range(2):
            spin[ik, :, sg * S:(sg + 1) * S, sg] = coll[2 * ik + sg]
            f_s[ik, sg * S:(sg + 1) * S] = f_c[2 * ik + sg]
    cs = P.project_fullgrid(sys_s, spin)
    cc = P.project_fullgrid(sys_c, coll)
    ns, ps, nbs = occ.occupations(sys_s, cs, f_s)
    nc, pc, nbc = occ.occupations(sys_c, cc, f_c)
    for I in range(len(sys_s.sites)):
        for sg in range(2):
            np.testing.assert_allclose(ns[I][sg, sg], nc[I][sg], atol=1e-14)
            np.testing.assert_allclose(ps[I][sg, sg], pc[I][sg], atol=1e-14)
        assert np.max(np.abs(ns[I][0, 1])) < 1e-15
