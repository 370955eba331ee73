"""Test helpers: turn a synthetic workload description into the oracle's
System.  Holds no arithmetic of the method."""

import numpy as np

from oracle.orbitals import Site, System


def to_system(cfg):
    sites = [Site(R=np.array(s["R"]), l=s["l"], zeta=s["zeta"], rc=s["rc"], species=s["species"],
                  zeta_dn=s.get("zeta_dn")) for s in cfg.sites]
    return System(cell=np.array(cfg.cell), ngrid=np.array(cfg.ngrid), sites=sites,
                  kpts=np.array(cfg.kpts), kweights=np.array(cfg.kweights), spin=cfg.spin)


def normwise(a, b):
    """max|a - b| / max|b| (0 when both vanish)."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if b.size else 0.0
    return num / den if den > 0 else num
