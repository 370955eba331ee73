"""One whole Hubbard step from the oracle's pieces.

project (Eq. occ_matrices brackets) -> n, N-bar, P-bar (Eqs. occ_matrices,
notation_Nbar, notation_Pbar) -> U-bar, J-bar (Eqs. ACBN0_U, ACBN0_J or
App. B) or a fixed U_eff (the empirical scheme, Sec. II) -> V, E_U
(Eqs. pot_V_U, E_Dudarev) -> V_U|psi>.  The real-time loop evaluates exactly
this step from the time-dependent states (Eq. pot_V_U_TD, adiabatic).
"""

import numpy as np

from . import acbn0, coulomb, occupations as occ, potential, projection


def site_tensors(system, spheres, method="fft"):
    g0 = coulomb.g0_box_average(system.h)
    return [coulomb.coulomb_tensor(system, s, sp, method=method, g0=g0)
            for s, sp in zip(system.sites, spheres)]


def hubbard_step(system, psi, f, spheres=None, tensors=None, ueff_fixed=None,
                 form="fullgrid", apply_block=None, on_block=None):
    """Return a dict with c, n, pbar, nbar, U, J, Ueff, status, V, EU, hpsi.

    ``ueff_fixed``: optional per-site list; a finite entry fixes that site's
    U_eff (empirical DFT+U), NaN/None computes it with ACBN0.
    ``apply_block``: evaluate V_U psi (sphere form) for that many state
    columns at a time, so that the complex output of a large workload need
    not be held whole; each block goes to ``on_block(s0, hpsi_block)`` and
    the returned hpsi is None.  The arithmetic of every column is the same.
    """
    if apply_block is not None and form != "sphere":
        raise ValueError("apply_block evaluates the sphere form of V_U psi")
    sps = spheres if spheres is not None else projection.all_spheres(system)
    if form == "fullgrid":
        c = projection.project_fullgrid(system, psi, sps)
    else:
        c = projection.project_sphere(system, psi, sps)
    n, pbar, nb = occ.occupations(system, c, f)
    nsites = len(system.sites)
    U = np.zeros(nsites)
    J = np.zeros(nsites)
    status = np.zeros(nsites, dtype=np.int64)
    Ueff = np.zeros(nsites)
    for I in range(nsites):
        fixed = None if ueff_fixed is None else ueff_fixed[I]
        if fixed is not None and np.isfinite(fixed):
            Ueff[I] = fixed
            U[I], J[I] = fixed, 0.0
            continue
        if system.spin == "spinor":
            U[I], J[I], status[I], _ = acbn0.uj_spinor(n[I], pbar[I], tensors[I])
        else:
            U[I], J[I], status[I], _ = acbn0.uj_collinear(
                occ.channels(system, n[I]), occ.channels(system, pbar[I]), tensors[I])
        Ueff[I] = U[I] - J[I]
    V = [potential.potential_matrix(system, Ueff[I], n[I]) for I in range(nsites)]
    EU = np.array([potential.energy(system, Ueff[I], n[I]) for I in range(nsites)])
    if apply_block is not None:
        hpsi = None
        for s0 in range(0, c.shape[2], apply_block):
            blk = apply_sphere(system, c[:, :, s0:s0 + apply_block], V, sps)
            if on_block is not None:
                on_block(s0, blk)
    elif form == "fullgrid":
        hpsi = potential.apply_fullgrid(system, c, V, sps)
    else:
        hpsi = apply_sphere(system, c, V, sps)
    return dict(c=c, n=n, pbar=pbar, nbar=nb, U=U, J=J, Ueff=Ueff, status=status,
                V=V, EU=EU, hpsi=hpsi)


def apply_sphere(system, c, V_list, spheres, G=None):
    """V_U|psi> scattered from the sphere points only (same result as
    potential.apply_fullgrid; pinned against it on small grids)."""
    from .orbitals import kphase
    B = potential.coefficients(system, c, V_list)
    off = projection.orbital_offsets(system)
    Gt = system.G if G is None else G
    tail = c.shape[2:]
    out = np.zeros((c.shape[0], Gt) + tail, dtype=np.complex128)
    for q in range(c.shape[0]):
        ik = q if system.spin == "spinor" else q // system.nspin
        k = system.kpts[ik]
        for I, sp in enumerate(spheres):
            w = np.conj(kphase(system, k, sp.n))[:, None] * sp.phi.T        # (P, L)
            blk = B[q, off[I]:off[I + 1]]
            contrib = np.tensordot(w, blk, axes=([1], [0]))                   # (P, S[, 2])
            np.add.at(out[q], sp.g, contrib)
    return out
