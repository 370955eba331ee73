"""ACBN0 U-bar and J-bar for one site.

Collinear (Sec. III, Eqs. ACBN0_U and ACBN0_J) and noncollinear (App. B).

Index reading of the numerators: the printed numerators
repeat m' and leave m''' free; they are read as
P-bar^alpha_{m m'} P-bar^beta_{m'' m'''} (m m'|m'' m''') for U and
P-bar^alpha_{m m'} P-bar^alpha_{m'' m'''} (m m'''|m'' m') for J, the same
index structure as the ACBN0 energy (Eq. HF_ACBN0) and as App. B.
Denominators use the bare occupations N^alpha_m = n^alpha_{mm} (Eq. ACBN0_J,
last line; App. B, last line).  The sums are formed term by term as written.

Degenerate denominators (below ``DEGEN``, e.g. one electron in one orbital)
are not treated by the paper; the value is then 0 and the status is 1.
"""

import numpy as np

DEGEN = 1e-12


def _num_U(Pa, Pb, T):
    return np.einsum("ab,cd,abcd->", Pa, Pb, T)


def _num_J(Pa, Pb, T):
    # sum P_{ab} P_{cd} (a d | c b)
    return np.einsum("ab,cd,adcb->", Pa, Pb, T)


def _ratio(num, den):
    if abs(den) < DEGEN:
        return 0.0, 1
    return num / den, 0


def uj_collinear(n, pbar, T):
    """n, pbar: (2, L, L) explicit spin channels.  Returns (U, J, status, imag).

    ``imag`` is the largest imaginary part met in the numerators (zero up to
    rounding for Hermitian P-bar and real orbitals)."""
    L = n.shape[-1]
    numU = sum(_num_U(pbar[a], pbar[b], T) for a in range(2) for b in range(2))
    numJ = sum(_num_J(pbar[a], pbar[a], T) for a in range(2))
    N = np.real(np.array([[n[a][m, m] for m in range(L)] for a in range(2)]))
    denJ = 0.0
    for a in range(2):
        for m in range(L):
            for mp in range(L):
                if m != mp:
                    denJ += N[a][m] * N[a][mp]
    denU = denJ
    for a in range(2):
        for m in range(L):
            for mp in range(L):
                denU += N[a][m] * N[1 - a][mp]
    U, sU = _ratio(numU.real, denU)
    J, sJ = _ratio(numJ.real, denJ)
    return U, J, max(sU, sJ), max(abs(numU.imag), abs(numJ.imag))


def uj_spinor(n, pbar, T):
    """n, pbar: (2, 2, L, L) indexed [sigma][sigma'][m][m'] (App. B)."""
    L = n.shape[-1]
    numU = sum(_num_U(pbar[s][s], pbar[t][t], T) for s in range(2) for t in range(2))
    numJ = sum(_num_J(pbar[s][t], pbar[t][s], T) for s in range(2) for t in range(2))
    Nd = lambda a, b, m: n[a][b][m, m]
    denU = 0.0 + 0.0j
    for s in range(2):
        for m in range(L):
            for mp in range(L):
                denU += Nd(s, s, m) * Nd(1 - s, 1 - s, mp)
                if m != mp:
                    denU += Nd(s, s, m) * Nd(s, s, mp)
        for m in range(L):
            denU -= Nd(s, 1 - s, m) * Nd(1 - s, s, m)
    denJ = 0.0 + 0.0j
    for s in range(2):
        for m in range(L):
            for mp in range(L):
                if m != mp:
                    denJ += Nd(s, s, m) * Nd(s, s, mp) + Nd(s, 1 - s, m) * Nd(1 - s, s, mp)
    U, sU = _ratio(numU.real, denU.real)
    J, sJ = _ratio(numJ.real, denJ.real)
    imag = max(abs(numU.imag), abs(numJ.imag), abs(denU.imag), abs(denJ.imag))
    return U, J, max(sU, sJ), imag
