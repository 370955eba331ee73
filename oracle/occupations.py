"""Occupation matrices n, renormalized occupations N-bar and matrices P-bar.

* n^{I,sigma}_{mm'} = sum_k w_k sum_n f_{nk}^sigma <psi|phi_m><phi_m'|psi>
  (Eq. occ_matrices).  With c_m = <phi_m|psi>, <psi|phi_m> = conj(c_m).
* N-bar_{psi} = sum over the sites I' of the same species as I and over their
  orbitals m of |<phi_{I',m}|psi>|^2 (Eq. notation_Nbar; "atoms of the same
  type" read as a caller-supplied species id per shell).
* P-bar^{I,sigma}_{mm'} = sum_{nk} w_k f_{nk} N-bar_{psi_nk} conj(c_m) c_m'
  (Eq. notation_Pbar).
* Spinors (App. A, App. B): n^{sigma sigma'}_{mm'} = sum w f conj(c^sigma_m)
  c^sigma'_m' with spin-independent orbitals; N-bar sums |c^sigma|^2 over both
  spin components (the orbital projector times the spin identity); P-bar is
  n with the extra N-bar weight.

Unpolarized runs hold one stored channel that stands for two identical spin
channels, each with occupations f in [0, 1].

Outputs (complex128):
* collinear/unpolarized: n[I] with shape (nchan, L, L), nchan = 1 or 2;
* spinor: n[I] with shape (2, 2, L, L) indexed [sigma][sigma'][m][m'].
* nbar[q][T][s] (collinear) / nbar[k][T][s] (spinor), float64.
"""

import numpy as np

from .projection import orbital_offsets


def nbar(system, c):
    off = orbital_offsets(system)
    nspec = 1 + max(s.species for s in system.sites)
    out = np.zeros((c.shape[0], nspec, c.shape[2]))
    for I, s in enumerate(system.sites):
        blk = c[:, off[I]:off[I + 1]]
        a2 = np.abs(blk) ** 2
        if system.spin == "spinor":
            a2 = a2.sum(axis=-1)
        out[:, s.species, :] += a2.sum(axis=1)
    return out


def _weights(system, f):
    """w_k f per stored state set, shape like f."""
    f = np.asarray(f, dtype=np.float64)
    if system.spin == "spinor":
        return system.kweights[:, None] * f
    wq = np.repeat(system.kweights, system.nspin)
    return wq[:, None] * f


def occupations(system, c, f, with_pbar=True):
    """Return (n, pbar, nbar) as lists over sites (see module docstring)."""
    off = orbital_offsets(system)
    wf = _weights(system, f)
    nb = nbar(system, c)
    n_out, p_out = [], []
    for I, s in enumerate(system.sites):
        blk = c[:, off[I]:off[I + 1]]                       # (q, L, S[, 2])
        wfn = wf * nb[:, s.species, :]
        if system.spin == "spinor":
            n = np.einsum("ks,kasx,kbsy->xyab", wf, np.conj(blk), blk)
            p = np.einsum("ks,kasx,kbsy->xyab", wfn, np.conj(blk), blk)
        else:
            ns = system.nspin
            n = np.zeros((ns, s.L, s.L), dtype=np.complex128)
            p = np.zeros((ns, s.L, s.L), dtype=np.complex128)
            for q in range(c.shape[0]):
                isp = q % ns
                n[isp] += (np.conj(blk[q]) * wf[q][None, :]) @ blk[q].T
                p[isp] += (np.conj(blk[q]) * wfn[q][None, :]) @ blk[q].T
        n_out.append(n)
        p_out.append(p)
    return n_out, (p_out if with_pbar else None), nb


def channels(system, n):
    """Expand one site's matrices to explicit spin channels.

    collinear: (2, L, L) unchanged; unpolarized: the single stored channel is
    duplicated to (2, L, L); spinor input is returned unchanged.
    """
    if system.spin == "unpolarized":
        return np.stack([n[0], n[0]])
    return n
