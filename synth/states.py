"""Seeded Kohn-Sham-like states and occupations.

Recipe:
* Random numbers come from ``numpy.random.default_rng(cfg.seed)`` on the host,
  drawn in a fixed order: for every state set q (k-point major, then spin),
  for every state: 8 Gaussian centres U(cell), widths U[0.5, 1.5] bohr and
  coefficients N(0, 1) (complex: independent real and imaginary parts;
  spinors: one coefficient per component).
* Each Gaussian is periodic through the minimum-image displacement; complex
  runs multiply by exp(i k.r), which makes every state a Bloch function
  psi(r + T) = exp(i k.T) psi(r).
* Each random part is normalized on the grid, then optional localized parts
  are added: Cartesian polynomials of the shell's degree times a Gaussian,
  centred on the atoms (generic localized functions, not the method's
  orbitals).  'afm' seeds the first states of each spin channel on one
  magnetic site; 'sites' adds a random combination over all sites.
* The states of every set are orthonormalized on the grid (dV metric) by
  CholQR applied twice.
Arrays are evaluated with torch on the requested device (the draws stay on
the host), in FP64 / complex128.  Layouts: psi[q][g][s] (q = k * nspin +
spin) or, for spinors, psi[k][g][s][sigma].
"""

import itertools

import numpy as np
import torch


def _grid_axes(cfg, device):
    h = [c / n for c, n in zip(cfg.cell, cfg.ngrid)]
    return [torch.arange(n, dtype=torch.float64, device=device) * hh for n, hh in zip(cfg.ngrid, h)]


def _grid_points(cfg, device):
    ax = _grid_axes(cfg, device)
    X, Y, Z = torch.meshgrid(*ax, indexing="ij")
    return torch.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], dim=1)


def _min_image(r, centre, cell):
    d = r - centre
    cellt = torch.tensor(cell, dtype=torch.float64, device=r.device)
    return d - cellt * torch.round(d / cellt)


def _dV(cfg):
    return float(np.prod([c / n for c, n in zip(cfg.cell, cfg.ngrid)]))


def _localized(cfg, r, centre, l, width, coeffs):
    """sum_a coeff_a * x^a0 y^a1 z^a2 (degree l) * exp(-|d|^2 / (2 w^2))."""
    d = _min_image(r, torch.tensor(centre, dtype=torch.float64, device=r.device), cfg.cell)
    mons = [e for e in itertools.product(range(l + 1), repeat=3) if sum(e) == l]
    poly = torch.zeros(r.shape[0], dtype=torch.float64, device=r.device)
    for cf, (a, b, c) in zip(coeffs, mons):
        poly = poly + float(cf) * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c
    return poly * torch.exp(-(d * d).sum(1) / (2.0 * width * width))


def _nmon(l):
    return (l + 1) * (l + 2) // 2


def _cholqr2(A, dV, rows=65536):
    """CholQR applied twice under the dV metric.  Only plain matrix products
    run on the device (in row blocks of a standard shape); the small Gram
    matrix is factorized and its triangular factor inverted on the host."""
    for _ in range(2):
        S = torch.zeros((A.shape[1], A.shape[1]), dtype=A.dtype, device=A.device)
        for r0 in range(0, A.shape[0], rows):
            blk = A[r0:r0 + rows]
            S += blk.conj().transpose(0, 1) @ blk
        S = (dV * S).cpu().numpy()
        S = 0.5 * (S + S.conj().T)
        R = np.linalg.cholesky(S).conj().T                      # S = R^H R, R upper triangular
        Rinv = np.linalg.solve(R, np.eye(R.shape[0], dtype=R.dtype))
        Rinv_d = torch.from_numpy(np.ascontiguousarray(Rinv)).to(A.device)
        for r0 in range(0, A.shape[0], rows):
            A[r0:r0 + rows] = A[r0:r0 + rows] @ Rinv_d
    return A


def make_states(cfg, device="cpu", chunk=32):
    """Return psi as a torch tensor (FP64 or complex128) on ``device``."""
    rng = np.random.default_rng(cfg.seed)
    r = _grid_points(cfg, device)
    G = r.shape[0]
    dV = _dV(cfg)
    ncomp = 2 if cfg.spin == "spinor" else 1
    cplx = cfg.is_complex
    dtype = torch.complex128 if cplx else torch.float64
    S = cfg.nstates
    nsets = cfg.nk if cfg.spin == "spinor" else cfg.nq
    shape = (nsets, G, S, 2) if ncomp == 2 else (nsets, G, S)
    psi = torch.empty(shape, dtype=dtype, device=device)
    loc = cfg.localized or {}
    for q in range(nsets):
        ik = q if cfg.spin == "spinor" else q // cfg.nspin
        isp = 0 if cfg.spin == "spinor" else q % cfg.nspin
        kvec = 2 * np.pi * np.asarray(cfg.kpts[ik]) / np.asarray(cfg.cell)
        # ---- random parts, drawn in order, evaluated in chunks of states
        for s0 in range(0, S, chunk):
            s1 = min(S, s0 + chunk)
            block = torch.zeros((G, s1 - s0, ncomp), dtype=dtype, device=device)
            for s in range(s0, s1):
                cen = rng.uniform(0.0, 1.0, size=(8, 3)) * np.asarray(cfg.cell)
                wid = rng.uniform(0.5, 1.5, size=8)
                co = rng.normal(size=(8, ncomp))
                if cplx:
                    co = co + 1j * rng.normal(size=(8, ncomp))
                for i in range(8):
                    d = _min_image(r, torch.tensor(cen[i], dtype=torch.float64, device=device), cfg.cell)
                    gss = torch.exp(-(d * d).sum(1) / (2.0 * wid[i] ** 2))
                    for x in range(ncomp):
                        block[:, s - s0, x] += complex(co[i, x]) * gss if cplx else float(co[i, x]) * gss
            nrm = torch.sqrt(dV * (block.abs() ** 2).sum(dim=(0, 2)))
            block = block / nrm[None, :, None]
            if ncomp == 2:
                psi[q, :, s0:s1, :] = block
            else:
                psi[q, :, s0:s1] = block[..., 0]
        # ---- localized parts
        kind = loc.get("kind")
        if kind == "afm":
            site = cfg.sites[loc["up_site"] if isp == 0 else loc["dn_site"]]
            for s in range(loc["nseed"]):
                cf = rng.normal(size=_nmon(site["l"]))
                f = _localized(cfg, r, site["R"], site["l"], loc["width"], cf)
                f = f / torch.sqrt(dV * (f * f).sum())
                psi[q, :, s] = f.to(dtype) + loc["noise"] * psi[q, :, s]
        elif kind == "sites":
            nloc = cfg.occ.get("nocc", S) if loc.get("nocc_only") else S
            basis = []
            for site in cfg.sites:
                cf = rng.normal(size=_nmon(site["l"]))
                f = _localized(cfg, r, site["R"], site["l"], loc["width"], cf)
                basis.append(f / torch.sqrt(dV * (f * f).sum()))
            Bm = torch.stack(basis, dim=1)                                    # (G, nsites)
            mix = rng.normal(size=(len(cfg.sites), nloc, ncomp))
            if cplx:
                mix = mix + 1j * rng.normal(size=mix.shape)
            mix = mix / np.sqrt(len(cfg.sites))
            for x in range(ncomp):
                add = Bm.to(dtype) @ torch.tensor(mix[..., x], dtype=dtype, device=device)
                if ncomp == 2:
                    psi[q, :, :nloc, x] += loc["amp"] * add
                else:
                    psi[q, :, :nloc] += loc["amp"] * add
        if cplx:
            ph = torch.exp(1j * (r @ torch.tensor(kvec, dtype=torch.float64, device=device)))
            psi[q] *= ph.view(G, 1, 1) if ncomp == 2 else ph.view(G, 1)
        # ---- orthonormalize this set
        if ncomp == 2:
            A = psi[q].permute(0, 2, 1).reshape(G * 2, S)
            A = _cholqr2(A, dV)
            psi[q] = A.reshape(G, 2, S).permute(0, 2, 1)
        else:
            psi[q] = _cholqr2(psi[q], dV)
    return psi


def make_occupations(cfg):
    """f per state set (numpy FP64): [nq][S] or, for spinors, [nk][S]."""
    rng = np.random.default_rng(1000 + cfg.seed)
    nsets = cfg.nk if cfg.spin == "spinor" else cfg.nq
    S = cfg.nstates
    occ = cfg.occ
    f = np.zeros((nsets, S))
    for q in range(nsets):
        if occ["kind"] == "aufbau":
            f[q, :occ["nocc"]] = 1.0
        else:
            eps = np.sort(rng.uniform(occ["emin"], occ["emax"], size=S))
            x = np.clip((eps - occ["mu"]) / occ["kT"], -700, 700)
            f[q] = 1.0 / (1.0 + np.exp(x))
    return f
