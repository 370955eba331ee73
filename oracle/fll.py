"""Noncollinear Hartree-Fock energy and the fully-localized-limit double
counting with magnetization (App. A).

Test infrastructure only (see oracle/__init__.py).

Per site, from the occupation blocks n^{st}_{ab} = sum w f conj(c^s_a) c^t_b
(Eq. occupation matrices of App. A; collinear runs have no spin-off-diagonal
blocks, unpolarized runs two equal diagonal blocks):

* N = sum_s sum_a n^{ss}_{aa}, the electrons in the localized shell;
* rho^{st} = sum_a n^{st}_{aa}, and the magnetization
  m_i = sum_{st} (sigma_i)_{st} rho^{st}, i.e. m_x = 2 Re rho^{ud},
  m_y = 2 Im rho^{ud}, m_z = rho^{uu} - rho^{dd};
* E_DC = U/2 N(N-1) - J/2 N(N/2-1) - J/4 m.m;
* E_ee, the Hartree-Fock energy of App. A written for occupation matrices
  diagonal in m, evaluated on the diagonal elements n^{st}_{aa}:
      U/2 sum_s sum_{a,b} n^{ss}_aa n^{s's'}_bb
    - U/2 sum_s sum_a n^{ss'}_aa n^{s's}_aa
    - J/2 sum_s sum_{a != b} n^{ss'}_aa n^{s's}_bb
    + (U-J)/2 sum_s sum_{a != b} n^{ss}_aa n^{ss}_bb,      s' = the other spin.

Reading: the paper writes m = Tr_s(sigma . rho) with its rho^{st}, whose
index order is the transpose of the usual spin density matrix; taken
literally that flips the sign of m_y.  m here is the physical magnetization
(a spinor along +y gives m_y = +1); E_DC depends on m.m only.
"""

import numpy as np


def spin_blocks(system, n):
    """One site's occupations as explicit (2, 2, L, L) spin blocks."""
    if system.spin == "spinor":
        return np.asarray(n)
    L = n.shape[-1]
    out = np.zeros((2, 2, L, L), dtype=np.complex128)
    out[0, 0] = n[0]
    out[1, 1] = n[0] if system.spin == "unpolarized" else n[1]
    return out


def moments(system, n):
    """(N, m) of one site: electron count and magnetization vector."""
    b = spin_blocks(system, n)
    rho = np.einsum("staa->st", b)
    N = float((rho[0, 0] + rho[1, 1]).real)
    m = np.array([2.0 * rho[0, 1].real, 2.0 * rho[0, 1].imag, (rho[0, 0] - rho[1, 1]).real])
    return N, m


def double_counting(N, m, U, J):
    return 0.5 * U * N * (N - 1.0) - 0.5 * J * N * (0.5 * N - 1.0) - 0.25 * J * float(np.dot(m, m))


def hf_energy(system, n, U, J):
    """E_ee of App. A on the m-diagonal elements of one site's blocks."""
    b = spin_blocks(system, n)
    d = np.einsum("staa->sta", b)                  # d[s, t, a] = n^{st}_aa
    L = d.shape[-1]
    off = ~np.eye(L, dtype=bool)
    E = 0.0
    for s in range(2):
        o = 1 - s
        E += 0.5 * U * np.sum(np.outer(d[s, s], d[o, o]))
        E -= 0.5 * U * np.sum(d[s, o] * d[o, s])
        E -= 0.5 * J * np.sum(np.outer(d[s, o], d[o, s])[off])
        E += 0.5 * (U - J) * np.sum(np.outer(d[s, s], d[s, s])[off])
    return float(np.real(E))
