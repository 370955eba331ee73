"""Hubbard forces through <phi|grad psi> (Sec. IV, the paper's own form).

Test infrastructure only (see oracle/__init__.py).

Sec. IV computes dn/dR from the derivatives of the states on the grid,
<phi_m|d psi/d r_i>, instead of differentiating the orbitals, to reduce the
egg-box effect.  In the continuum d c/d R_i = -<d phi/d r_i|psi> =
+<phi|d psi/d r_i> (integration by parts, up to the surface term of the
cutoff at r_c), so the force of forces.py holds with d = -<phi|D_i psi>:

    F_i = 2 Re sum w f sum_ab V_ab conj(-e_{a,i}) c_b,   e = <phi|D_i psi>.

D_i is the 4th-order central difference on the cell grid (the paper gives
no stencil; 4th order is the usual real-space choice), applied to the
Bloch extension of psi: a neighbour that leaves the cell along axis i is
psi at the folded point times exp(i k_i a_i) per crossing.
"""

import numpy as np

from .forces import forces_analytic
from .projection import project_sphere

# first derivative, offsets -2..2 (divided by h)
STENCIL = {-2: 1.0 / 12.0, -1: -2.0 / 3.0, 1: 2.0 / 3.0, 2: -1.0 / 12.0}


def _kset(system, q):
    return q if system.spin == "spinor" else q // system.nspin


def fd_gradient(system, psi):
    """D_i psi for i = 0, 1, 2: array shaped (3,) + psi.shape."""
    psi = np.asarray(psi)
    Nx, Ny, Nz = (int(n) for n in system.ngrid)
    h = np.asarray(system.cell, dtype=np.float64) / np.asarray(system.ngrid)
    out = np.zeros((3,) + psi.shape, dtype=np.complex128)
    for q in range(psi.shape[0]):
        k = 2 * np.pi * np.asarray(system.kpts[_kset(system, q)], dtype=np.float64) / np.asarray(system.cell)
        grid = psi[q].reshape((Nx, Ny, Nz) + psi.shape[2:])
        for i, N in enumerate((Nx, Ny, Nz)):
            acc = np.zeros(grid.shape, dtype=np.complex128)
            idx = np.arange(N)
            for m, cm in STENCIL.items():
                j = idx + m
                wraps = np.floor_divide(j, N)                      # lattice crossings along i
                src = np.take(grid, j - wraps * N, axis=i)
                ph = np.exp(1j * k[i] * system.cell[i] * wraps)
                shape = [1] * grid.ndim
                shape[i] = N
                acc += cm * src * ph.reshape(shape)
            out[i, q] = (acc / h[i]).reshape(psi[q].shape)
    return out


def state_gradient_projections(system, psi, spheres):
    """e[q][j][i][s] (spinor: e[k][j][i][s][sigma]) = <phi_j|D_i psi>."""
    D = fd_gradient(system, psi)
    return np.stack([project_sphere(system, D[i], spheres) for i in range(3)], axis=2)


def forces_state_gradient(system, c, e, V_list, f):
    """F[I][i] from c, e = <phi|D psi> and V (the Sec. IV form)."""
    return forces_analytic(system, c, -e, V_list, f)
