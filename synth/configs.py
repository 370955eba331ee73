"""Geometry and run parameters of the five workloads, full size and reduced.

The five workloads are synthetic systems shaped like those the paper studies
(a single transition-metal d shell; a NiO-like antiferromagnetic rock-salt
oxide with k-points; many uneven p/d/f sites in a real-time loop;
noncollinear spinors in a layered hexagonal-like cell; a many-site cell for
forces).  No dataset is involved.  Reduced ("small") variants keep the same
structure at sizes the CPU oracle handles in seconds while still spanning
several kernel tiles and a ragged tail of states.
"""

from dataclasses import dataclass, field

import numpy as np

CONFIG_NAMES = ("gamma_d", "nio_afm", "rt_batched", "spinor_layers", "forces_fcc")


@dataclass
class Config:
    name: str
    cell: tuple
    ngrid: tuple
    sites: list                      # dicts: R, l, zeta, rc, species
    kpts: np.ndarray
    kweights: np.ndarray
    spin: str                        # 'unpolarized' | 'collinear' | 'spinor'
    is_complex: bool
    nstates: int
    seed: int
    occ: dict = field(default_factory=dict)
    localized: dict = field(default_factory=dict)
    extra: dict = field(default_factory=dict)

    @property
    def nk(self):
        return len(self.kpts)

    @property
    def nspin(self):
        return 2 if self.spin == "collinear" else 1

    @property
    def nq(self):
        return self.nk * self.nspin

    @property
    def G(self):
        return int(np.prod(self.ngrid))


def _site(R, l, zeta, rc, species):
    return dict(R=np.asarray(R, dtype=np.float64), l=int(l), zeta=float(zeta), rc=float(rc), species=int(species))


def gamma_d(small=False):
    """Single d shell at the centre of a 10 bohr cube, Gamma point, real states."""
    n = 40
    return Config(
        name="gamma_d", cell=(10.0, 10.0, 10.0), ngrid=(n, n, n),
        sites=[_site((5.0, 5.0, 5.0), 2, 2.0, 4.0, 0)],
        kpts=np.zeros((1, 3)), kweights=np.ones(1), spin="unpolarized", is_complex=False,
        nstates=16, seed=1, occ=dict(kind="aufbau", nocc=8))


def nio_afm(small=False):
    """NiO-like collinear antiferromagnet: 2 Ni d + 2 O p sites, 2x2x2 k."""
    a = 8.35
    n = 24 if small else 48
    kk = [(x, y, z) for x in (-0.25, 0.25) for y in (-0.25, 0.25) for z in (-0.25, 0.25)]
    if small:
        kk = kk[:2]
    sites = [_site((0, 0, 0), 2, 2.2, 4.2, 0), _site((a / 2, a / 2, a / 2), 2, 2.2, 4.2, 0),
             _site((a / 2, a / 2, 0), 1, 1.6, 3.5, 1), _site((0, 0, a / 2), 1, 1.6, 3.5, 1)]
    return Config(
        name="nio_afm", cell=(a, a, a), ngrid=(n, n, n), sites=sites,
        kpts=np.array(kk), kweights=np.full(len(kk), 1.0 / len(kk)), spin="collinear",
        is_complex=True, nstates=(40 if small else 64), seed=2,
        occ=dict(kind="fermi", kT=0.01, mu=0.0, emin=-1.0, emax=0.5, nlow=5),
        localized=dict(kind="afm", up_site=0, dn_site=1, nseed=5, noise=0.1, width=0.8))


def rt_batched(small=False):
    """Uneven p/d/f sites on a simple-cubic lattice, real-time loop (Gamma, real)."""
    rng = np.random.default_rng(3)
    per = 2 if small else 4
    spacing = 9.0
    h = 0.3
    L = per * spacing
    n = int(round(L / h))
    offset = rng.uniform(0.0, h, size=3)
    lattice = [(i, j, k) for i in range(per) for j in range(per) for k in range(per)]
    even = [p for p in lattice if sum(p) % 2 == 0]
    nf = max(1, len(even) // 4)
    perm = rng.permutation(len(even))
    f_set = set(tuple(even[i]) for i in perm[:nf])
    sites = []
    for p in lattice:
        base = np.array(p, dtype=np.float64) * spacing + offset
        if sum(p) % 2 == 1:
            sites.append(_site(base, 1, 1.6, 3.5, 0))
        elif tuple(p) in f_set:
            sites.append(_site(base, 3, 2.4, 5.5, 2))
        else:
            jit = rng.uniform(-0.3, 0.3, size=3)
            sites.append(_site(base + jit, 2, 2.0, 4.5, 1))
    return Config(
        name="rt_batched", cell=(L, L, L), ngrid=(n, n, n), sites=sites,
        kpts=np.zeros((1, 3)), kweights=np.ones(1), spin="unpolarized", is_complex=False,
        nstates=(200 if small else 1024), seed=3,
        occ=dict(kind="aufbau", nocc=(100 if small else 512)),
        localized=dict(kind="sites", amp=0.3, width=1.0, nocc_only=True),
        extra=dict(steps=100, angle=1e-3))


def spinor_layers(small=False):
    """Noncollinear spinors: 7 layers with ABC in-plane stacking, 5 p + 2 d."""
    a = 7.8
    b = 13.5
    c = 28.0
    ng = (16, 28, 56) if small else (32, 56, 112)
    inplane = [(0.0, 0.0), (a / 2, a / (2 * np.sqrt(3))), (0.0, a / np.sqrt(3))]
    sites = []
    for t in range(7):
        x, y = inplane[t % 3]
        R = (x + 0.1, y + 0.1, 4.0 * t + 2.0 + 0.1)
        if t in (2, 5):
            sites.append(_site(R, 2, 2.0, 4.0, 1))
        else:
            sites.append(_site(R, 1, 1.4, 4.0, 0))
    kk = [(x, y, 0.0) for x in (-0.25, 0.25) for y in (-0.25, 0.25)]
    if small:
        kk = kk[:2]
    return Config(
        name="spinor_layers", cell=(a, b, c), ngrid=ng, sites=sites,
        kpts=np.array(kk), kweights=np.full(len(kk), 1.0 / len(kk)), spin="spinor",
        is_complex=True, nstates=(40 if small else 256), seed=4,
        occ=dict(kind="fermi", kT=0.01, mu=0.0, emin=-1.0, emax=0.5, nlow=0),
        localized=dict(kind="sites", amp=0.3, width=1.0, nocc_only=False))


def forces_fcc(small=False):
    """32 d sites on a 2x2x2 fcc supercell (Gamma, real), for forces."""
    rng = np.random.default_rng(5)
    a = 14.4
    ncell = 1 if small else 2
    basis = [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]
    sites = []
    for i in range(ncell):
        for j in range(ncell):
            for k in range(ncell):
                for bvec in basis:
                    R = (np.array([i, j, k], dtype=np.float64) + np.array(bvec)) * a + 0.15
                    R = R + rng.uniform(-0.3, 0.3, size=3)
                    sites.append(_site(R, 2, 2.0, 4.5, 0))
    L = ncell * a
    n = 48 if small else 96
    return Config(
        name="forces_fcc", cell=(L, L, L), ngrid=(n, n, n), sites=sites,
        kpts=np.zeros((1, 3)), kweights=np.ones(1), spin="unpolarized", is_complex=False,
        nstates=(96 if small else 512), seed=5,
        occ=dict(kind="aufbau", nocc=(48 if small else 256)),
        localized=dict(kind="sites", amp=0.3, width=1.0, nocc_only=True))


_MAKERS = dict(gamma_d=gamma_d, nio_afm=nio_afm, rt_batched=rt_batched,
               spinor_layers=spinor_layers, forces_fcc=forces_fcc)


def make_config(name, small=False, **overrides):
    cfg = _MAKERS[name](small=small)
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg
