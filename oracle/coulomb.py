"""On-site Coulomb integrals (mm'|m''m''') evaluated on the real-space grid.

Paper passages followed:
* Sec. III: ACBN0 needs only a reduced set of Coulomb integrals, and the
  implementation evaluates them directly from the orbitals on the real-space
  grid (not from a three-Gaussian fit).
* App. B, notation for (m m' sigma | m'' m''' sigma'): the double integral of
  phi_m* phi_m'(r1) phi_m''* phi_m'''(r2) / |r1 - r2|.

Discretisation (readings where the paper is silent):
* Free-space (isolated) kernel even in periodic cells: the integrals are
  single-centre, over the unfolded sphere points of one site.
* T[a,b,c,d] = dV^2 sum_{p,p'} rho_ab(p) K(p - p') rho_cd(p'),
  rho_ab = phi_a phi_b (real orbitals), K(r) = 1/|r| for r != 0 and
  K(0) = G0 = the average of 1/r over one grid cell centred on the origin.
* ``hockney_potential`` performs the convolution with a zero-padded FFT
  (padding 2B >= 2B-1 makes the circular convolution equal the linear one);
  ``direct_potential`` is the O(N^2) double sum it must reproduce.

Continuum reference (used only to pin the grid result as h -> 0):
Slater integrals F^k of the truncated, continuum-normalized radial function
and real Gaunt coefficients, T = sum_k 4 pi/(2k+1) F^k sum_q G(ab,kq) G(cd,kq).
"""

import numpy as np
from scipy import integrate

from .harmonics import real_ylm


# ----------------------------------------------------------------- G(0) term
def g0_box_average(h):
    """(1 / (hx hy hz)) * integral of 1/|r| over the cell [-h/2, h/2]^3.

    The octant box [0,a]x[0,b]x[0,c] is split into three pyramids with apex
    at the origin, one per far face; on the face x = a the substitution
    y = x u, z = x v turns the pyramid integral into
    (a^2 / 2) * int_0^{b/a} int_0^{c/a} du dv / sqrt(1 + u^2 + v^2).
    """
    hx, hy, hz = (float(v) for v in h)
    half = [hx / 2, hy / 2, hz / 2]
    total = 0.0
    for ax in range(3):
        a = half[ax]
        b, c = [half[i] for i in range(3) if i != ax]
        val, _ = integrate.dblquad(lambda v, u: 1.0 / np.sqrt(1.0 + u * u + v * v),
                                   0.0, b / a, 0.0, c / a, epsabs=1e-15, epsrel=1e-14)
        total += 0.5 * a * a * val
    return 8.0 * total / (hx * hy * hz)


# --------------------------------------------------------------- convolution
def _kernel_on_padded(shape, h, g0):
    axes = []
    for M, hh in zip(shape, h):
        o = np.arange(M)
        o = np.where(o < M // 2, o, o - M)
        axes.append(o * hh)
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    K = np.empty_like(r)
    nz = r > 0
    K[nz] = 1.0 / r[nz]
    K[~nz] = g0
    return K


def hockney_potential(rho, h, g0):
    """v(p) = dV * sum_p' K(p - p') rho(p') on a box, for a stack of densities.

    rho: array (Bx, By, Bz, ndens).  Returns the same shape.
    """
    B = rho.shape[:3]
    M = tuple(2 * b for b in B)
    dV = float(np.prod(h))
    Kf = np.fft.fftn(_kernel_on_padded(M, h, g0))
    out = np.empty(rho.shape)
    for i in range(rho.shape[3]):
        pad = np.zeros(M)
        pad[:B[0], :B[1], :B[2]] = rho[..., i]
        v = np.fft.ifftn(np.fft.fftn(pad) * Kf).real
        out[..., i] = dV * v[:B[0], :B[1], :B[2]]
    return out


def direct_potential(ijk, rho, h, g0):
    """O(N^2) double sum on an explicit point list.

    ijk: integer coordinates (P, 3); rho: (P, ndens).  Returns (P, ndens).
    """
    pos = ijk.astype(np.float64) * np.asarray(h, dtype=np.float64)
    diff = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=2))
    K = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), g0)
    return float(np.prod(h)) * (K @ rho)


# ------------------------------------------------------------- site tensors
def unfolded_ijk(system, sphere):
    N = system.ngrid
    ix = sphere.g // (N[1] * N[2])
    iy = (sphere.g // N[2]) % N[1]
    iz = sphere.g % N[2]
    return np.stack([ix, iy, iz], axis=1) + sphere.n * N[None, :]


def pair_densities(L, phi):
    """rho_ab(p) = phi_a(p) phi_b(p) for all (a, b), shape (P, L*L)."""
    return np.stack([phi[a] * phi[b] for a in range(L) for b in range(L)], axis=1)


def coulomb_tensor(system, site, sphere, method="fft", g0=None):
    """T[a,b,c,d] = (ab|cd) for one site, shape (L, L, L, L)."""
    h = system.h
    if g0 is None:
        g0 = g0_box_average(h)
    L = site.L
    rho = pair_densities(L, sphere.phi)
    ijk = unfolded_ijk(system, sphere)
    if method == "direct":
        v = direct_potential(ijk, rho, h, g0)
    elif method == "fft":
        lo = ijk.min(axis=0)
        B = tuple(int(v) for v in (ijk.max(axis=0) - lo + 1))
        box = np.zeros(B + (rho.shape[1],))
        loc = ijk - lo
        box[loc[:, 0], loc[:, 1], loc[:, 2]] = rho
        vb = hockney_potential(box, h, g0)
        v = vb[loc[:, 0], loc[:, 1], loc[:, 2]]
    else:
        raise ValueError(method)
    T = system.dV * (rho.T @ v)                      # (L*L, L*L): [ab][cd]
    return T.reshape(L, L, L, L)


# ---------------------------------------------------- continuum reference
def slater_Fk(l, zeta, rc, k):
    """F^k for R(r) ~ r^l exp(-zeta r) on [0, rc], normalized on [0, rc]."""
    P = lambda r: r ** (2 * l + 2) * np.exp(-2.0 * zeta * r)
    norm, _ = integrate.quad(P, 0.0, rc, epsabs=0, epsrel=2e-14, limit=200)

    def inner(r1):
        a, _ = integrate.quad(lambda r2: P(r2) * r2 ** k, 0.0, r1, epsabs=0, epsrel=1e-13, limit=200)
        return a

    outer, _ = integrate.quad(lambda r1: P(r1) * r1 ** (-(k + 1)) * inner(r1) if r1 > 0 else 0.0,
                              0.0, rc, epsabs=0, epsrel=1e-12, limit=200)
    return 2.0 * outer / (norm * norm)


def real_gaunt_table(l, kmax):
    """G[a, b, k, q] = integral of Y_{l a} Y_{l b} Y_{k q} over the sphere
    (a, b index m = -l..l, q index -k..k), by product quadrature exact for
    these degrees."""
    xg, wg = np.polynomial.legendre.leggauss(40)
    nphi = 80
    ph = 2 * np.pi * np.arange(nphi) / nphi
    CT, PH = np.meshgrid(xg, ph, indexing="ij")
    ST = np.sqrt(1 - CT * CT)
    x, y, z = ST * np.cos(PH), ST * np.sin(PH), CT
    W = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :])
    Ys = {(ll, m): real_ylm(ll, m, x, y, z) for ll in set([l] + list(range(kmax + 1))) for m in range(-ll, ll + 1)}
    L = 2 * l + 1
    G = np.zeros((L, L, kmax + 1, 2 * kmax + 1))
    for a in range(L):
        for b in range(L):
            for k in range(kmax + 1):
                for q in range(-k, k + 1):
                    G[a, b, k, q + k] = np.sum(W * Ys[(l, a - l)] * Ys[(l, b - l)] * Ys[(k, q)])
    return G


def continuum_tensor(l, zeta, rc):
    L = 2 * l + 1
    G = real_gaunt_table(l, 2 * l)
    T = np.zeros((L, L, L, L))
    for k in range(0, 2 * l + 1):
        Fk = slater_Fk(l, zeta, rc, k)
        Gk = G[:, :, k, :2 * k + 1]
        T += 4 * np.pi / (2 * k + 1) * Fk * np.einsum("abq,cdq->abcd", Gk, Gk)
    return T
