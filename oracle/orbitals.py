"""Localized orbitals on atom-centred spheres, with Bloch sums over images.

Paper passages followed:
* Sec. II, discussion after Eq. pot_V_U: the localized orbitals are atomic-like
  functions (radial part times a spherical harmonic) represented on spherical
  sub-grids centred on the atoms; in a periodic cell a sphere may cross the
  box border, and the points outside the box are mapped back onto the regular
  grid with a phase (Fig. 1, "sketch").
* Sec. II, sphere-radius discussion: the sphere is truncated at a radius r_c.
* Eq. occ_matrices: the projections are <phi_{I,m}|psi_{nk}>.

Readings where the paper is silent:
* The radial part is a Slater-type r^l exp(-zeta r) (the paper's come from
  pseudopotentials); phi_m(r) = N_m exp(-zeta |r|) S_lm(r) with S_lm the real
  solid harmonic.
* Sphere membership is inclusive, |d|^2 <= r_c^2, where d is computed
  canonically: h_i = cell_i / N_i, x_i = j_i * h_i for the *unfolded* integer
  grid coordinate j_i, d_i = x_i - R_i, |d|^2 = (d_x^2 + d_y^2) + d_z^2, all in
  FP64 with no fused operations.
* N_m normalizes each function on the grid over the sphere points:
  dV * sum_p phi_m(p)^2 = 1 (no cross-m orthogonalization; the paper assumes
  orthogonality, Sec. III).
* Bloch convention: psi_k(r + T) = exp(i k.T) psi_k(r).  The Bloch orbital on
  the cell grid is Phi_{m,k}(r_g) = sum_T exp(-i k.T) phi_m(r_g + T - R), so
  that <Phi_{m,k}|psi> = dV sum_p exp(+i k.T_p) phi_m(p) psi(g(p)).
* Grid index g = (ix * Ny + iy) * Nz + iz; r_g = (ix hx, iy hy, iz hz).
"""

from dataclasses import dataclass, field

import numpy as np

from .harmonics import solid_harmonic, solid_harmonic_grad


@dataclass
class Site:
    R: np.ndarray
    l: int
    zeta: float
    rc: float
    species: int = 0
    zeta_dn: float = None        # spin-down exponent of spinor orbitals (spinorb.py); None: zeta

    @property
    def L(self):
        return 2 * self.l + 1


@dataclass
class System:
    cell: np.ndarray                     # (3,) orthorhombic cell lengths, bohr
    ngrid: np.ndarray                    # (3,) grid points per axis
    sites: list
    kpts: np.ndarray = field(default_factory=lambda: np.zeros((1, 3)))   # reduced k
    kweights: np.ndarray = field(default_factory=lambda: np.ones(1))
    spin: str = "unpolarized"            # 'unpolarized' | 'collinear' | 'spinor'

    def __post_init__(self):
        self.cell = np.asarray(self.cell, dtype=np.float64)
        self.ngrid = np.asarray(self.ngrid, dtype=np.int64)
        self.kpts = np.atleast_2d(np.asarray(self.kpts, dtype=np.float64))
        self.kweights = np.asarray(self.kweights, dtype=np.float64)
        for s in self.sites:
            s.R = np.asarray(s.R, dtype=np.float64)

    @property
    def h(self):
        return self.cell / self.ngrid

    @property
    def dV(self):
        h = self.h
        return float(h[0] * h[1] * h[2])

    @property
    def G(self):
        return int(np.prod(self.ngrid))

    @property
    def nk(self):
        return self.kpts.shape[0]

    @property
    def nspin(self):
        """Number of independent spin channels stored for collinear modes."""
        return 2 if self.spin == "collinear" else 1

    @property
    def nq(self):
        """Number of (k, spin) state sets for collinear layouts."""
        return self.nk * self.nspin


@dataclass
class Sphere:
    """Unfolded sphere points of one site: grid index g, image n (T = n*cell),
    displacement d = r_p - R, orbital values phi (L, P)."""
    g: np.ndarray
    n: np.ndarray
    d: np.ndarray
    phi: np.ndarray
    norms: np.ndarray


def _axis_candidates(system, site, axis, brute):
    N = int(system.ngrid[axis])
    a = float(system.cell[axis])
    R = float(site.R[axis])
    nlo = int(np.floor((R - site.rc) / a)) - 1
    nhi = int(np.floor((R + site.rc) / a)) + 1
    out = []
    for n in range(nlo, nhi + 1):
        ix = np.arange(N, dtype=np.int64)
        if not brute:
            h = a / N
            x = (ix + n * N) * h
            ix = ix[(x >= R - site.rc - h) & (x <= R + site.rc + h)]
        if ix.size:
            out.append((n, ix))
    return out


def sphere_points(system, site, brute=False):
    """Enumerate the unfolded sphere points of ``site``.

    For every lattice image n (per axis) the cell grid indices ix are shifted to
    unfolded coordinates j = ix + n*N and tested for |d|^2 <= r_c^2.  With
    ``brute=True`` every grid point of every image is tested (slow; used to pin
    the bounding-box restriction on small grids).
    Returns (g, n, d) sorted by (g, n).
    """
    h = system.cell / system.ngrid
    Nx, Ny, Nz = (int(v) for v in system.ngrid)
    cand = [_axis_candidates(system, site, ax, brute) for ax in range(3)]
    gs, ns, ds = [], [], []
    rc2 = site.rc * site.rc
    for nx, ix in cand[0]:
        dx = (ix + nx * Nx) * h[0] - site.R[0]
        for ny, iy in cand[1]:
            dy = (iy + ny * Ny) * h[1] - site.R[1]
            for nz, iz in cand[2]:
                dz = (iz + nz * Nz) * h[2] - site.R[2]
                DX, DY, DZ = np.meshgrid(dx, dy, dz, indexing="ij")
                d2 = (DX * DX + DY * DY) + DZ * DZ
                mask = d2 <= rc2
                if not mask.any():
                    continue
                IX, IY, IZ = np.meshgrid(ix, iy, iz, indexing="ij")
                g = (IX[mask] * Ny + IY[mask]) * Nz + IZ[mask]
                gs.append(g)
                ns.append(np.tile(np.array([nx, ny, nz], dtype=np.int64), (g.size, 1)))
                ds.append(np.stack([DX[mask], DY[mask], DZ[mask]], axis=1))
    if not gs:
        return np.zeros(0, np.int64), np.zeros((0, 3), np.int64), np.zeros((0, 3))
    g = np.concatenate(gs)
    n = np.concatenate(ns)
    d = np.concatenate(ds)
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0], g))
    return g[order], n[order], d[order]


def radial_angular(site, d):
    """Unnormalized chi_m(d) = exp(-zeta |d|) S_lm(d), shape (L, P)."""
    r = np.sqrt(np.sum(d * d, axis=1))
    rad = np.exp(-site.zeta * r)
    return np.stack([rad * solid_harmonic(site.l, m, d[:, 0], d[:, 1], d[:, 2])
                     for m in range(-site.l, site.l + 1)])


def radial_angular_grad(site, d):
    """Gradient of chi_m with respect to the point r (i.e. d), shape (L, 3, P).

    grad[exp(-zeta r) S] = exp(-zeta r) (grad S - zeta (d / r) S); the second
    term vanishes at r = 0 for l >= 1, and is taken as 0 there for l = 0.
    """
    r = np.sqrt(np.sum(d * d, axis=1))
    rad = np.exp(-site.zeta * r)
    safe = np.where(r > 0, r, 1.0)
    out = []
    for m in range(-site.l, site.l + 1):
        S = solid_harmonic(site.l, m, d[:, 0], d[:, 1], d[:, 2])
        gS = solid_harmonic_grad(site.l, m, d[:, 0], d[:, 1], d[:, 2])
        unit = np.where(r > 0, 1.0 / safe, 0.0) * d.T
        out.append(rad * (gS - site.zeta * unit * S))
    return np.stack(out)


def build_sphere(system, site, brute=False, R_eval=None, norms=None):
    """Sphere of ``site``: points from the reference position, orbital values
    evaluated at ``R_eval`` (default: site.R) with normalization ``norms``
    (default: computed here so that dV * sum_p phi^2 = 1).

    Passing R_eval/norms gives the frozen-membership, frozen-normalization
    orbitals used for position derivatives (Sec. IV; see forces.py).
    """
    g, n, d = sphere_points(system, site, brute=brute)
    if R_eval is not None:
        d = d + (site.R - np.asarray(R_eval, dtype=np.float64))
    chi = radial_angular(site, d)
    if norms is None:
        norms = 1.0 / np.sqrt(system.dV * np.sum(chi * chi, axis=1))
    return Sphere(g=g, n=n, d=d, phi=chi * norms[:, None], norms=norms)


def kphase(system, k_red, n):
    """exp(i k.T) for T = n * cell, k = 2 pi k_red / cell (per axis)."""
    return np.exp(2j * np.pi * (np.asarray(n, dtype=np.float64) @ np.asarray(k_red, dtype=np.float64)))


def bloch_orbitals(system, site, k_red, sphere=None):
    """Phi_{m,k}(r_g) on the whole cell grid, complex (L, G).

    Each unfolded sphere point p contributes exp(-i k.T_p) phi_m(p) at its
    folded grid point g(p); points that fold onto the same g add.
    """
    sp = sphere if sphere is not None else build_sphere(system, site)
    out = np.zeros((site.L, system.G), dtype=np.complex128)
    ph = np.conj(kphase(system, k_red, sp.n))
    for m in range(site.L):
        np.add.at(out[m], sp.g, ph * sp.phi[m])
    return out
