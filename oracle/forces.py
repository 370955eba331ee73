"""Hubbard forces and gradients of E_U.

Sec. IV: F = -dE_U/dR = -sum (dE_U/dn_mm') (dn_mm'/dR), with
dE_U/dn_mm' = (U_eff/2)(delta_mm' - 2 n_m'm) (the printed U is the effective
U; U_eff held fixed, Sec. III).  The occupations depend on R through the
projections; the primary form here differentiates the orbitals:
c(R) = dV sum_p exp(i k.T_p) phi(r_p - R) psi(g(p)) with sphere membership,
images and normalization frozen at the reference position, so
dc/dR = -d, d = dV sum_p exp(i k.T_p) (grad phi)(p) psi(g(p)) and

    F_i = 2 Re sum_{k,sigma} w_k sum_n f_n sum_ab V_ab conj(d_{a,i}) c_b.

(The paper's printed dn/dR formulas are garbled in their indices; this form
is the exact derivative of the discrete E_U and is checked against central
finite differences below.  The alternative through <phi|grad psi>, which
the paper uses, is in stencil.py.)

Adjoint: dE_U/dpsi*(g) = dV w_k f_n (V_U psi)(g) (Eq. minimization); for
unpolarized runs, which count the stored channel twice, both results double.
"""

import numpy as np

from .orbitals import build_sphere, kphase, radial_angular_grad
from .projection import orbital_offsets, project_sphere
from .occupations import occupations, _weights
from .potential import coefficients, energy, potential_matrix


def gradient_projections(system, psi, spheres):
    """d[q][j][i][s] (collinear) or d[k][j][i][s][sigma] (spinor)."""
    out = []
    for ik in range(system.nk):
        k = system.kpts[ik]
        qs = [ik] if system.spin == "spinor" else [ik * system.nspin + i for i in range(system.nspin)]
        for q in qs:
            blocks = []
            for site, sp in zip(system.sites, spheres):
                gphi = radial_angular_grad(site, sp.d) * sp.norms[:, None, None]    # (L, 3, P)
                w = gphi * kphase(system, k, sp.n)[None, None, :] * system.dV
                rows = psi[q][sp.g]
                if system.spin == "spinor":
                    blocks.append(np.einsum("aip,psx->aisx", w, rows))
                else:
                    blocks.append(np.einsum("aip,ps->ais", w, rows))
            out.append(np.concatenate(blocks))
    return np.stack(out)


def forces_analytic(system, c, d, V_list, f):
    """F[I][i] from projections c, gradient projections d and potentials V."""
    off = orbital_offsets(system)
    B = coefficients(system, c, V_list)
    wf = _weights(system, f)
    degen = 2.0 if system.spin == "unpolarized" else 1.0
    F = np.zeros((len(system.sites), 3))
    for I, _ in enumerate(system.sites):
        sl = slice(off[I], off[I + 1])
        for i in range(3):
            if system.spin == "spinor":
                val = np.einsum("ks,kasx,kasx->", wf, np.conj(d[:, sl, i]), B[:, sl])
            else:
                val = np.einsum("qs,qas,qas->", wf, np.conj(d[:, sl, i]), B[:, sl])
            F[I, i] = degen * 2.0 * val.real
    return F


def energy_at(system, psi, f, ueffs, spheres):
    c = project_sphere(system, psi, spheres)
    n, _, _ = occupations(system, c, f, with_pbar=False)
    return sum(energy(system, u, nn) for u, nn in zip(ueffs, n))


def fd_force(system, psi, f, ueffs, I, i, delta=1e-4):
    """-(E(R + delta e_i) - E(R - delta e_i)) / (2 delta), frozen sphere."""
    ref = [build_sphere(system, s) for s in system.sites]
    vals = []
    for sgn in (+1.0, -1.0):
        R = system.sites[I].R.copy()
        R[i] += sgn * delta
        sps = list(ref)
        sps[I] = build_sphere(system, system.sites[I], R_eval=R, norms=ref[I].norms)
        vals.append(energy_at(system, psi, f, ueffs, sps))
    return -(vals[0] - vals[1]) / (2 * delta)


def psi_gradient(system, psi, f, ueffs, spheres, apply_fn):
    """dE_U/dpsi* as an array shaped like psi, from V_U psi (``apply_fn``)."""
    c = project_sphere(system, psi, spheres)
    n, _, _ = occupations(system, c, f, with_pbar=False)
    V = [potential_matrix(system, u, nn) for u, nn in zip(ueffs, n)]
    hpsi = apply_fn(system, c, V, spheres)
    wf = _weights(system, f)
    degen = 2.0 if system.spin == "unpolarized" else 1.0
    if system.spin == "spinor":
        return degen * system.dV * hpsi * wf[:, None, :, None]
    return degen * system.dV * hpsi * wf[:, None, :]
