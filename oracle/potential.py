"""Hubbard potential V_U|psi> and the Dudarev energy E_U.

* E_U = sum_I U_eff/2 sum_{m,sigma} (n_mm - sum_m' n_mm' n_m'm)
  (Eq. E_Dudarev); noncollinear: U_eff/2 [sum_{sigma,m} n^{ss}_mm -
  sum_{mm' ss'} n^{ss'}_{mm'} n^{s's}_{m'm}] (App. A, final equation).
* V_U|psi> = sum_I sum_{mm'} V_mm' |phi_m><phi_m'|psi> (Eq. pot_V_U).

Transpose reading: the potential is the functional
derivative of E_U with respect to psi* (Eq. minimization).  With
n_mm' = <psi|phi_m><phi_m'|psi> this derivative gives
V_ab = U_eff (delta_ab / 2 - n_ba), i.e. the transpose of the printed
n_ab; the two agree for real states and differ for complex k-states.
Noncollinear: V^{ss'}_{ab} = U_eff (delta_ss' delta_ab / 2 - n^{s's}_{ba}),
derived from the App. A energy the same way.  ACBN0 uses the same potential
with U_eff = U-bar - J-bar held fixed (Sec. III, last paragraph before the
tables).
"""

import numpy as np

from .projection import bloch_matrix, orbital_offsets


def potential_matrix(system, ueff, n):
    """V for one site from its occupation matrices (layout as in
    occupations.py: (nchan, L, L) or (2, 2, L, L))."""
    L = n.shape[-1]
    eye = np.eye(L)
    if system.spin == "spinor":
        V = np.zeros((2, 2, L, L), dtype=np.complex128)
        for s in range(2):
            for t in range(2):
                V[s, t] = ueff * ((0.5 * eye if s == t else 0.0) - n[t, s].T)
        return V
    return np.stack([ueff * (0.5 * eye - n[c].T) for c in range(n.shape[0])])


def energy(system, ueff, n):
    """E_U of one site (explicit spin channels: unpolarized counts twice)."""
    if system.spin == "spinor":
        L = n.shape[-1]
        N = np.block([[n[0, 0], n[0, 1]], [n[1, 0], n[1, 1]]])
        val = np.trace(N) - np.trace(N @ N)
        return 0.5 * ueff * val.real
    chans = [n[0], n[0]] if system.spin == "unpolarized" else [n[0], n[1]]
    val = sum(np.trace(m) - np.trace(m @ m) for m in chans)
    return 0.5 * ueff * val.real


def coefficients(system, c, V_list):
    """B = V c per site: the coefficients of |phi_a> in V_U|psi>."""
    off = orbital_offsets(system)
    B = np.zeros_like(c, dtype=np.complex128)
    for I, _ in enumerate(system.sites):
        sl = slice(off[I], off[I + 1])
        V = V_list[I]
        for q in range(c.shape[0]):
            if system.spin == "spinor":
                for s in range(2):
                    B[q, sl, :, s] = sum(V[s, t] @ c[q, sl, :, t] for t in range(2))
            else:
                B[q, sl] = V[q % system.nspin] @ c[q, sl]
    return B


def apply_fullgrid(system, c, V_list, spheres=None):
    """(V_U psi)(r_g) = sum_a Phi_{a,k}(r_g) B_a, same layout as psi."""
    B = coefficients(system, c, V_list)
    out = []
    for ik in range(system.nk):
        Phi = bloch_matrix(system, system.kpts[ik], spheres)
        if system.spin == "spinor":
            out.append(np.stack([Phi.T @ B[ik][..., s] for s in range(2)], axis=-1))
        else:
            for isp in range(system.nspin):
                q = ik * system.nspin + isp
                out.append(Phi.T @ B[q])
    return np.stack(out)
