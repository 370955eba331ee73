"""Projections c_{I,m}(n,k,sigma) = <phi_{I,m,k}|psi_{n,k,sigma}>.

Follows Eq. occ_matrices (the brackets <phi|psi> it is built from) with the
Bloch orbitals of ``orbitals.bloch_orbitals`` (Sec. II and Fig. 1: phase for
sphere points that cross the box border).

Two forms:
* ``project_fullgrid``: the plain definition, dV * sum over every cell grid
  point of conj(Phi_{m,k}(r_g)) psi(r_g).  Dense and slow; the reference.
* ``project_sphere``: the same sum restricted to the sphere points where
  Phi is non-zero, dV * sum_p exp(+i k.T_p) phi_m(p) psi(g(p)).  Pinned
  against ``project_fullgrid`` on small grids; used for large cases.

State layouts (FP64 / complex128 numpy arrays):
* collinear / unpolarized: psi[q][g][s], q = ik * nspin + ispin;
* spinor: psi[k][g][s][sigma].
Orbital index j runs over (site, m) in site order, m = -l..l.
"""

import numpy as np

from .orbitals import bloch_orbitals, build_sphere, kphase


def all_spheres(system):
    return [build_sphere(system, s) for s in system.sites]


def orbital_offsets(system):
    off = [0]
    for s in system.sites:
        off.append(off[-1] + s.L)
    return off


def bloch_matrix(system, k_red, spheres=None):
    """All Bloch orbitals of the system stacked, complex (J, G)."""
    sps = spheres if spheres is not None else all_spheres(system)
    return np.concatenate([bloch_orbitals(system, s, k_red, sp) for s, sp in zip(system.sites, sps)])


def project_fullgrid(system, psi, spheres=None):
    """c[q][j][s] (collinear) or c[k][j][s][sigma] (spinor), complex128."""
    psi = np.asarray(psi)
    out = []
    for ik in range(system.nk):
        Phi = bloch_matrix(system, system.kpts[ik], spheres)
        A = np.conj(Phi) * system.dV
        if system.spin == "spinor":
            out.append(np.stack([A @ psi[ik][..., sg] for sg in range(2)], axis=-1))
        else:
            for isp in range(system.nspin):
                out.append(A @ psi[ik * system.nspin + isp])
    return np.stack(out)


def project_sphere(system, psi, spheres=None, cols=None):
    """Same result as ``project_fullgrid`` from the sphere points only.

    ``cols`` optionally restricts the state columns (for sampled checks on
    very large inputs); psi may then be any array indexable as psi[q][g][s].
    """
    sps = spheres if spheres is not None else all_spheres(system)
    out = []
    for ik in range(system.nk):
        k = system.kpts[ik]
        qs = [ik] if system.spin == "spinor" else [ik * system.nspin + i for i in range(system.nspin)]
        for q in qs:
            blocks = []
            for sp in sps:
                rows = np.asarray(psi[q][sp.g] if cols is None else psi[q][sp.g][:, cols])
                w = (kphase(system, k, sp.n)[None, :] * sp.phi) * system.dV      # (L, P)
                if system.spin == "spinor":
                    blocks.append(np.stack([w @ rows[..., sg] for sg in range(2)], axis=-1))
                else:
                    blocks.append(w @ rows)
            out.append(np.concatenate(blocks))
    return np.stack(out)
