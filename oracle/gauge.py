"""Velocity-gauge Hubbard operator and the DFT+U current correction (Sec. V).

Test infrastructure only (see oracle/__init__.py).

With a uniform vector potential A(t), Sec. V replaces the operator by its
gauge-transformed form V^A = exp(-i A.r) V_U exp(+i A.r).  On the sphere
points this means that the bra of every localized orbital picks up
exp(+i A.r_p) at its unfolded point r_p = R_I + d_p, next to the Bloch phase
exp(i k.T_p) of Fig. 1:

    c^A_m = dV sum_p exp(i k.T_p) exp(i A.r_p) phi_m(p) psi(g(p)),
    (V^A psi)(g) = sum_{p: g(p) = g} exp(-i k.T_p) exp(-i A.r_p) sum_m phi_m(p) B_m,

with B = V c^A and V built from the occupations of c^A as at A = 0.

Current correction.  As printed, -1/2 sum w f <psi|[r, V^A]|psi> + c.c.
vanishes identically: [r, V^A] is anti-Hermitian, so its expectation is
imaginary and cancels against its conjugate.  The reading used here
restores the factor i of the velocity operator v = i[H, r]:

    J_U = sum_{k,sigma} w_k sum_n f_n <psi| i [V^A, r] |psi>
        = sum w f <psi| dV^A/dA |psi>          (n and U_eff held fixed),

because dV^A/dA = -i [r, V^A].  In projections, with the position moments
rho_{a,i} = dV sum_p exp(i k.T_p) exp(i A.r_p) (d_p)_i phi_a(p) psi(g(p))
about the site centre (a constant shift of r cancels in the commutator),

    J_U,i = 2 sum w f Im sum_a conj(rho_{a,i}) B_a,

the forces' contraction with Im in place of Re.  Unpolarized runs count the
stored channel twice, as in the energy.
"""

import numpy as np

from .occupations import _weights
from .orbitals import kphase
from .potential import coefficients
from .projection import orbital_offsets


def gauge_phase(system, k_red, site, sphere, A):
    """exp(i k.T_p) exp(i A.r_p) at every unfolded point of one sphere."""
    A = np.asarray(A, dtype=np.float64)
    r = site.R[None, :] + sphere.d
    return kphase(system, k_red, sphere.n) * np.exp(1j * (r @ A))


def _sets(system, ik):
    return [ik] if system.spin == "spinor" else [ik * system.nspin + i for i in range(system.nspin)]


def project_gauge(system, psi, spheres, A):
    """c^A, same layout as ``projection.project_sphere``."""
    out = []
    for ik in range(system.nk):
        k = system.kpts[ik]
        for q in _sets(system, ik):
            blocks = []
            for site, sp in zip(system.sites, spheres):
                w = gauge_phase(system, k, site, sp, A)[None, :] * sp.phi * system.dV     # (L, P)
                rows = np.asarray(psi[q][sp.g])
                if system.spin == "spinor":
                    blocks.append(np.stack([w @ rows[..., x] for x in range(2)], axis=-1))
                else:
                    blocks.append(w @ rows)
            out.append(np.concatenate(blocks))
    return np.stack(out)


def moment_projections(system, psi, spheres, A):
    """rho[q][j][i][s] (spinor: rho[k][j][i][s][sigma]): the position moments
    about each site centre, with the gauge and Bloch phases."""
    out = []
    for ik in range(system.nk):
        k = system.kpts[ik]
        for q in _sets(system, ik):
            blocks = []
            for site, sp in zip(system.sites, spheres):
                ph = gauge_phase(system, k, site, sp, A)
                w = sp.phi[:, None, :] * sp.d.T[None, :, :] * ph[None, None, :] * system.dV    # (L, 3, P)
                rows = np.asarray(psi[q][sp.g])
                if system.spin == "spinor":
                    blocks.append(np.einsum("aip,psx->aisx", w, rows))
                else:
                    blocks.append(np.einsum("aip,ps->ais", w, rows))
            out.append(np.concatenate(blocks))
    return np.stack(out)


def apply_gauge(system, c, V_list, spheres, A):
    """V^A psi on the cell grid (same layout as psi) from c = c^A."""
    B = coefficients(system, c, V_list)
    off = orbital_offsets(system)
    nsets = c.shape[0]
    shape = (nsets, system.G) + c.shape[2:]
    out = np.zeros(shape, dtype=np.complex128)
    for ik in range(system.nk):
        k = system.kpts[ik]
        for q in _sets(system, ik):
            for I, (site, sp) in enumerate(zip(system.sites, spheres)):
                ph = np.conj(gauge_phase(system, k, site, sp, A))                           # (P,)
                blk = B[q, off[I]:off[I + 1]]                                              # (L, S[, 2])
                contrib = np.tensordot(sp.phi * ph[None, :], blk, axes=([0], [0]))          # (P, S[, 2])
                np.add.at(out[q], sp.g, contrib)
    return out


def current(system, c, rho, V_list, f):
    """J_U per site, shape (n_sites, 3): 2 sum w f Im sum_a conj(rho_a) B_a."""
    off = orbital_offsets(system)
    B = coefficients(system, c, V_list)
    wf = _weights(system, f)
    degen = 2.0 if system.spin == "unpolarized" else 1.0
    J = np.zeros((len(system.sites), 3))
    for I, _ in enumerate(system.sites):
        sl = slice(off[I], off[I + 1])
        for i in range(3):
            if system.spin == "spinor":
                val = np.einsum("ks,kasx,kasx->", wf, np.conj(rho[:, sl, i]), B[:, sl])
            else:
                val = np.einsum("qs,qas,qas->", wf, np.conj(rho[:, sl, i]), B[:, sl])
            J[I, i] = degen * 2.0 * val.imag
    return J


def expectation(system, c, V_list, f):
    """sum w f <psi|V|psi> = sum w f sum_ab conj(c_a) V_ab c_b (real; both
    spin channels for unpolarized runs)."""
    B = coefficients(system, c, V_list)
    wf = _weights(system, f)
    degen = 2.0 if system.spin == "unpolarized" else 1.0
    if system.spin == "spinor":
        val = np.einsum("ks,kasx,kasx->", wf, np.conj(c), B)
    else:
        val = np.einsum("qs,qas,qas->", wf, np.conj(c), B)
    return degen * val.real
