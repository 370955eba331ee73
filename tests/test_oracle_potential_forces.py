"""Pins for oracle.potential, oracle.forces and oracle.step (CPU).

* E_U >= 0 for occupation eigenvalues in [0, 1] and E_U = 0 for an idempotent
  occupation matrix (Eq. E_Dudarev).
* V_U is the derivative of E_U (Eq. minimization): a central finite
  difference of E_U along a random direction of complex k-point states
  equals 2 Re sum dV w f conj(dpsi) V_U psi.  This fixes the transpose
  reading of V (the printed n_ab instead of n_ba fails it).
* Noncollinear: the same finite-difference identity for spinors; single
  component spinors reproduce the collinear E_U and V_U psi; a global SU(2)
  rotation leaves E_U invariant and rotates V_U psi covariantly.
* V_U is Hermitian: <chi|V_U psi> = conj <psi|V_U chi>.
* The sphere scatter form of V_U psi equals the full-grid form.
* Forces (Sec. IV): the analytic <grad phi|psi> force equals a central
  finite difference of E_U in the atom position (frozen sphere membership
  and normalization), and vanishes by symmetry for an orbital-shaped state on
  a grid-symmetric centre.
"""

import numpy as np
import pytest

from oracle import forces as FO
from oracle import occupations as occ
from oracle import potential as POT
from oracle import projection as P
from oracle import step as ST
from oracle.orbitals import Site, System, build_sphere
from tests.helpers import normwise


def _system(spin="collinear", kpts=((0.25, -0.25, 0.5), (0.0, 0.25, 0.0))):
    return System(cell=[6.0, 6.5, 7.0], ngrid=[12, 13, 14],
                  sites=[Site(R=[0.3, 6.2, 3.3], l=2, zeta=1.6, rc=3.4, species=0),
                         Site(R=[3.1, 3.0, 0.5], l=1, zeta=1.3, rc=2.8, species=1)],
                  kpts=np.array(kpts), kweights=np.full(len(kpts), 1.0 / len(kpts)), spin=spin)


def _states(sys_, S, seed, spinor=False):
    rng = np.random.default_rng(seed)
    sps = P.all_spheres(sys_)
    out = []
    for ik in range(sys_.nk):
        Phi = P.bloch_matrix(sys_, sys_.kpts[ik], sps)
        nsets = 1 if spinor else sys_.nspin
        for _ in range(nsets):
            if spinor:
                A = rng.normal(size=(sys_.G * 2, S)) + 1j * rng.normal(size=(sys_.G * 2, S))
                loc = np.concatenate([Phi.T, Phi.T]) @ (rng.normal(size=(Phi.shape[0], S)) + 1j * rng.normal(size=(Phi.shape[0], S)))
                Q, _ = np.linalg.qr(0.2 * A + loc)
                out.append((Q / np.sqrt(sys_.dV)).reshape(2, sys_.G, S).transpose(1, 2, 0))
            else:
                A = rng.normal(size=(sys_.G, S)) + 1j * rng.normal(size=(sys_.G, S))
                loc = Phi.T @ (rng.normal(size=(Phi.shape[0], S)) + 1j * rng.normal(size=(Phi.shape[0], S)))
                Q, _ = np.linalg.qr(0.2 * A + loc)
                out.append(Q / np.sqrt(sys_.dV))
    return np.stack(out), sps


def _energy(sys_, psi, f, ueffs, sps):
    c = P.project_fullgrid(sys_, psi, sps)
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    return sum(POT.energy(sys_, u, nn) for u, nn in zip(ueffs, n))


def test_energy_sign_and_idempotent_zero():
    sys_ = _system()
    L = 5
    rng = np.random.default_rng(1)
    for _ in range(5):
        A = rng.normal(size=(L, L)) + 1j * rng.normal(size=(L, L))
        Hm = A @ A.conj().T
        n = Hm / np.linalg.eigvalsh(Hm).max()
        assert POT.energy(sys_, 0.3, np.stack([n, 0.5 * n])) >= 0
    Q, _ = np.linalg.qr(rng.normal(size=(L, L)) + 1j * rng.normal(size=(L, L)))
    proj = Q[:, :2] @ Q[:, :2].conj().T
    assert abs(POT.energy(sys_, 0.7, np.stack([proj, np.eye(L)]))) < 1e-14


@pytest.mark.parametrize("spin", ["collinear", "spinor", "unpolarized"])
def test_potential_is_energy_derivative(spin):
    kp = ((0.0, 0.0, 0.0),) if spin == "unpolarized" else ((0.25, -0.25, 0.5), (0.0, 0.25, 0.0))
    sys_ = _system(spin=spin, kpts=kp)
    S = 5
    psi, sps = _states(sys_, S, 3, spinor=(spin == "spinor"))
    if spin == "unpolarized":
        psi = psi.real.copy()
    rng = np.random.default_rng(8)
    nsets = psi.shape[0]
    f = rng.uniform(0.2, 1.0, size=(nsets, S))
    ueffs = [0.37, 0.21]
    d = rng.normal(size=psi.shape) + (1j * rng.normal(size=psi.shape) if np.iscomplexobj(psi) else 0)
    eps = 1e-6
    fd = (_energy(sys_, psi + eps * d, f, ueffs, sps) - _energy(sys_, psi - eps * d, f, ueffs, sps)) / (2 * eps)
    grad = FO.psi_gradient(sys_, psi, f, ueffs, sps, POT.apply_fullgrid)       # dE/dpsi*
    an = 2 * np.real(np.sum(np.conj(d) * grad))
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an))
    assert abs(an) > 1e-3
    if spin == "collinear":
        # the printed (untransposed) reading of V gives a different, wrong slope
        c = P.project_fullgrid(sys_, psi, sps)
        n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
        Vbad = [np.stack([u * (0.5 * np.eye(m.shape[-1]) - m[ch]) for ch in range(2)]) for u, m in zip(ueffs, n)]
        hbad = POT.apply_fullgrid(sys_, c, Vbad, sps)
        wq = np.repeat(sys_.kweights, 2)[:, None] * f
        bad = 2 * np.real(np.sum(np.conj(d) * sys_.dV * hbad * wq[:, None, :]))
        assert abs(bad - fd) > 1e3 * abs(fd - an)


def test_potential_hermitian_and_sphere_form():
    sys_ = _system()
    psi, sps = _states(sys_, 4, 5)
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 1, size=(sys_.nq, 4))
    c = P.project_fullgrid(sys_, psi, sps)
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, u, nn) for u, nn in zip([0.3, 0.5], n)]
    h_full = POT.apply_fullgrid(sys_, c, V, sps)
    h_sph = ST.apply_sphere(sys_, c, V, sps)
    assert normwise(h_sph, h_full) < 1e-13
    # Hermiticity with V fixed: <chi|V psi> = conj <psi|V chi>
    chi, _ = _states(sys_, 4, 6)
    cc = P.project_fullgrid(sys_, chi, sps)
    h_chi = POT.apply_fullgrid(sys_, cc, V, sps)
    lhs = np.einsum("qgs,qgs->qs", np.conj(chi), h_full)
    rhs = np.conj(np.einsum("qgs,qgs->qs", np.conj(psi), h_chi))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_spinor_reduces_to_collinear_and_su2_covariance():
    sc = _system(spin="collinear")
    ss = _system(spin="spinor")
    S = 4
    coll, sps = _states(sc, S, 12)
    rng = np.random.default_rng(3)
    f_c = rng.uniform(0, 1, size=(sc.nq, S))
    spin = np.zeros((ss.nk, ss.G, 2 * S, 2), dtype=np.complex128)
    f_s = np.zeros((ss.nk, 2 * S))
    for ik in range(ss.nk):
        for sg in range(2):
            spin[ik, :, sg * S:(sg + 1) * S, sg] = coll[2 * ik + sg]
            f_s[ik, sg * S:(sg + 1) * S] = f_c[2 * ik + sg]
    ueff = [0.4, 0.25]
    oc = ST.hubbard_step(sc, coll, f_c, sps, ueff_fixed=ueff)
    os_ = ST.hubbard_step(ss, spin, f_s, sps, ueff_fixed=ueff)
    np.testing.assert_allclose(os_["EU"], oc["EU"], atol=1e-14)
    for ik in range(ss.nk):
        for sg in range(2):
            np.testing.assert_allclose(os_["hpsi"][ik][:, sg * S:(sg + 1) * S, sg], oc["hpsi"][2 * ik + sg], atol=1e-13)
    # SU(2): psi -> W psi for every spinor
    a, b = rng.normal(size=2) + 1j * rng.normal(size=2)
    W = np.array([[a, -np.conj(b)], [b, np.conj(a)]]) / np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    rot = np.einsum("st,kgnt->kgns", W, spin)
    orot = ST.hubbard_step(ss, rot, f_s, sps, ueff_fixed=ueff)
    np.testing.assert_allclose(orot["EU"], os_["EU"], atol=1e-13)
    np.testing.assert_allclose(orot["hpsi"], np.einsum("st,kgnt->kgns", W, os_["hpsi"]), atol=1e-12)


def test_forces_match_finite_differences():
    sys_ = System(cell=[9.0, 9.0, 9.0], ngrid=[30, 30, 30],
                  sites=[Site(R=[2.03, 4.41, 4.62], l=2, zeta=2.0, rc=3.2),
                         Site(R=[6.71, 4.52, 4.38], l=1, zeta=1.5, rc=2.9)],
                  kpts=[[0.0, 0.0, 0.0]], kweights=[1.0], spin="unpolarized")
    rng = np.random.default_rng(21)
    sps = P.all_spheres(sys_)
    Phi = P.bloch_matrix(sys_, np.zeros(3), sps).real
    S = 6
    A = 0.2 * rng.normal(size=(sys_.G, S)) + Phi.T @ rng.normal(size=(Phi.shape[0], S))
    Q, _ = np.linalg.qr(A)
    psi = (Q / np.sqrt(sys_.dV))[None]
    f = np.array([[1, 1, 1, 0.5, 0.2, 0.0]])
    ueffs = [0.31, 0.17]
    c = P.project_sphere(sys_, psi, sps)
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, u, nn) for u, nn in zip(ueffs, n)]
    d = FO.gradient_projections(sys_, psi, sps)
    F = FO.forces_analytic(sys_, c, d, V, f)
    assert np.max(np.abs(F)) > 1e-3
    for I in range(2):
        for i in range(3):
            fd = FO.fd_force(sys_, psi, f, ueffs, I, i, delta=1e-4)
            assert abs(fd - F[I, i]) < 1e-7 * np.max(np.abs(F)) + 1e-10


def test_force_vanishes_by_symmetry():
    sys_ = System(cell=[8, 8, 8], ngrid=[32, 32, 32], sites=[Site(R=[4, 4, 4], l=2, zeta=2.0, rc=3.0)])
    sps = P.all_spheres(sys_)
    Phi = P.bloch_matrix(sys_, np.zeros(3), sps).real
    psi = Phi[[0, 2]].T[None].copy()
    psi[0, :, 1] *= 0.999                       # two orbital-shaped states
    f = np.array([[1.0, 0.6]])
    c = P.project_sphere(sys_, psi, sps)
    n, _, _ = occ.occupations(sys_, c, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, 0.4, n[0])]
    F = FO.forces_analytic(sys_, c, FO.gradient_projections(sys_, psi, sps), V, f)
    assert np.max(np.abs(F)) < 1e-14


def test_step_with_column_blocks_matches_whole_step():
    """The column-blocked apply of the oracle step (used to bound host memory
    on the 1024-state workload) hands over exactly the columns of the
    full-grid V_U psi, block by block, ragged last block included."""
    sys_ = _system()
    S = 7
    psi, sps = _states(sys_, S, 21)
    rng = np.random.default_rng(8)
    f = rng.uniform(0, 1, size=(sys_.nq, S))
    ueff = [0.35, 0.2]
    whole = ST.hubbard_step(sys_, psi, f, sps, ueff_fixed=ueff)
    got = np.zeros_like(whole["hpsi"])
    seen = []

    def keep(s0, blk):
        seen.append((s0, blk.shape[2]))
        got[:, :, s0:s0 + blk.shape[2]] = blk

    part = ST.hubbard_step(sys_, psi, f, sps, ueff_fixed=ueff, form="sphere", apply_block=3, on_block=keep)
    assert part["hpsi"] is None
    assert seen == [(0, 3), (3, 3), (6, 1)]
    assert normwise(got, whole["hpsi"]) < 1e-13
    for I in range(len(sps)):
        assert normwise(part["n"][I], whole["n"][I]) < 1e-13, I
    for k in ("Ueff", "EU"):
        assert normwise(part[k], whole[k]) < 1e-13, k
