"""Spin-dependent localized orbitals of noncollinear runs (App. A).

Test infrastructure only (see oracle/__init__.py).

App. A allows the localized basis to be spinors: the projection of the spin
component sigma of a state uses that component's orbital,
n^{st}_{ab} = sum w f conj(<phi^s_a|psi^s>) <phi^t_b|psi^t>.  Here a site may
carry a second Slater exponent ``zeta_dn`` for the spin-down component (same
l, same sphere radius and points; each component is normalized on the grid
on its own, as in orbitals.build_sphere).  A site without one uses the same
orbital for both components, which is the spin-independent case.

Everything after the projection (occupations, U_eff, V, E_U) is unchanged;
the apply builds component sigma of V_U psi from phi^sigma:
(V_U psi)^s(r_g) = sum_a Phi^s_{a,k}(r_g) B^s_a, B^s = sum_t V^{st} c^t
(potential.coefficients).  U_eff is given (the empirical scheme): App. B
writes ACBN0 for spin-independent orbitals.  The forces (Sec. IV) and the
current (Sec. V) keep their forms with the gradient and position-moment
projections of each component's orbital (forces.forces_analytic,
gauge.current on the spinor layout).
"""

import numpy as np

from .orbitals import Site, System, kphase
from .potential import coefficients
from .projection import all_spheres, bloch_matrix, project_fullgrid, project_sphere


def component_systems(system):
    """One-component systems (spin-up orbitals, spin-down orbitals) on the
    same grid and k-points; each projects a (nk, G, S) component array."""
    def one(dn):
        sites = [Site(R=s.R, l=s.l, zeta=(s.zeta_dn if dn and s.zeta_dn is not None else s.zeta), rc=s.rc,
                      species=s.species) for s in system.sites]
        return System(cell=system.cell, ngrid=system.ngrid, sites=sites, kpts=system.kpts,
                      kweights=system.kweights, spin="unpolarized")
    return one(False), one(True)


def project_spin(system, psi, form="fullgrid"):
    """c[k][j][s][sigma] = <phi^sigma_{j,k}|psi^sigma_{s,k}>."""
    out = []
    for sg, comp in enumerate(component_systems(system)):
        x = np.asarray(psi)[..., sg]
        out.append(project_fullgrid(comp, x) if form == "fullgrid" else project_sphere(comp, x, all_spheres(comp)))
    return np.stack(out, axis=-1)


def apply_spin(system, c, V_list, form="fullgrid"):
    """V_U psi with the spin-dependent orbitals, layout of psi (spinor)."""
    B = coefficients(system, c, V_list)
    comps = component_systems(system)
    out = np.zeros((system.nk, system.G) + c.shape[2:], dtype=np.complex128)
    for sg, comp in enumerate(comps):
        sps = all_spheres(comp)
        for ik in range(system.nk):
            if form == "fullgrid":
                Phi = bloch_matrix(comp, system.kpts[ik], sps)                 # (J, G)
                out[ik, :, :, sg] = Phi.T @ B[ik, :, :, sg]
            else:
                off = 0
                for site, sp in zip(comp.sites, sps):
                    ph = np.conj(kphase(comp, system.kpts[ik], sp.n))
                    blk = B[ik, off:off + site.L, :, sg]
                    np.add.at(out[ik, :, :, sg], sp.g, (sp.phi * ph[None, :]).T @ blk)
                    off += site.L
    return out


def _per_component(system, psi, fn):
    """Stack fn(component system, component states, its spheres) over the two
    spin components on a last axis."""
    out = []
    for sg, comp in enumerate(component_systems(system)):
        out.append(fn(comp, np.asarray(psi)[..., sg], all_spheres(comp)))
    return np.stack(out, axis=-1)


def gradient_projections_spin(system, psi):
    """d[k][j][i][s][sigma] = <grad phi^sigma_j|psi^sigma_s> (forces.py form)."""
    from .forces import gradient_projections
    return _per_component(system, psi, gradient_projections)


def moment_projections_spin(system, psi, A=(0.0, 0.0, 0.0)):
    """rho[k][j][i][s][sigma]: position moments of phi^sigma (gauge.py form)."""
    from .gauge import moment_projections
    return _per_component(system, psi, lambda comp, x, sps: moment_projections(comp, x, sps, A))


def project_gauge_spin(system, psi, A):
    """c^A[k][j][s][sigma] with the orbital of each spin component."""
    from .gauge import project_gauge
    return _per_component(system, psi, lambda comp, x, sps: project_gauge(comp, x, sps, A))


def apply_gauge_spin(system, c, V_list, A):
    """V^A psi with the spin-dependent orbitals (gauge.py's apply, each
    component scattered through its own orbital), from c = c^A."""
    from .gauge import gauge_phase
    B = coefficients(system, c, V_list)
    out = np.zeros((system.nk, system.G) + c.shape[2:], dtype=np.complex128)
    for sg, comp in enumerate(component_systems(system)):
        sps = all_spheres(comp)
        for ik in range(system.nk):
            off = 0
            for site, sp in zip(comp.sites, sps):
                ph = np.conj(gauge_phase(comp, system.kpts[ik], site, sp, A))
                blk = B[ik, off:off + site.L, :, sg]
                np.add.at(out[ik, :, :, sg], sp.g, (sp.phi * ph[None, :]).T @ blk)
                off += site.L
    return out


def state_gradient_projections_spin(system, psi):
    """e[k][j][i][s][sigma] = <phi^sigma_j|D_i psi^sigma_s> (stencil.py form)."""
    from .stencil import state_gradient_projections
    return _per_component(system, psi, state_gradient_projections)
