"""CPU test of the library's state-gradient work list (no GPU, no kernel).

tests/host/stencil_tables.cpp is compiled with g++ against the library's
host sphere builder (sphere.cpp); it checks every chunk index against its
buffer and sums the dilated-sphere table against the states as the
projection kernels do.  The result must equal the oracle's -<phi|D psi>
(4th-order differences of the states, then the plain sphere projection):
spheres that reach past half the cell, sites next to the cell faces, an s
shell next to p/d/f shells, generic k-points, and the spin-down orbitals'
table of a context with spin-dependent orbitals.  Every case runs both
with a plain build of the checker and with one under host AddressSanitizer
and UndefinedBehaviorSanitizer."""

import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from oracle import projection as P
from oracle import stencil as SG
from oracle.orbitals import Site, System
from tests.helpers import normwise

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_08935_amd", "csrc")

CASES = [
    ([6.0, 6.5, 7.0], [12, 13, 14], [Site(R=[0.3, 6.2, 3.3], l=2, zeta=1.6, rc=3.4),
                                     Site(R=[3.1, 3.0, 0.5], l=1, zeta=1.3, rc=2.8, species=1)], [0.25, -0.25, 0.5]),
    ([5.0, 5.0, 5.0], [10, 10, 10], [Site(R=[0.0, 0.0, 0.0], l=3, zeta=1.2, rc=4.1),
                                     Site(R=[2.5, 4.99, 0.01], l=0, zeta=1.0, rc=1.3, species=1)], [0.1, 0.37, -0.2]),
    ([8.0, 8.0, 8.0], [40, 40, 40], [Site(R=[0.05, 7.97, 4.0], l=2, zeta=1.6, rc=2.0)], [0.0, 0.0, 0.0]),
    ([6.0, 6.5, 7.0], [12, 13, 14], [Site(R=[0.3, 6.2, 3.3], l=2, zeta=1.6, rc=3.4, zeta_dn=2.3),
                                     Site(R=[3.1, 3.0, 0.5], l=1, zeta=1.3, rc=2.8, species=1)], [0.25, -0.25, 0.5]),
]


# the checker is built plain and with host AddressSanitizer and
# UndefinedBehaviorSanitizer (any report aborts it with a non-zero status)
SANITIZE = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def checker(request, tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("stencil") / "stencil_tables")
    extra = SANITIZE if request.param == "sanitized" else []
    subprocess.run([gxx, "-O2", "-ffp-contract=off", "-std=c++17", *extra, "-I", os.path.join(ROOT, "include"), "-I",
                    CSRC, os.path.join(ROOT, "tests", "host", "stencil_tables.cpp"), os.path.join(CSRC, "sphere.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("case", range(len(CASES)))
def test_stencil_tables_match_oracle(checker, tmp_path, case):
    cell, ngrid, sites, k = CASES[case]
    sys_ = System(cell=cell, ngrid=ngrid, sites=sites, kpts=np.array([k]), kweights=np.ones(1), spin="unpolarized")
    S = 3
    rng = np.random.default_rng(case)
    psi = rng.normal(size=(1, sys_.G, S)) + 1j * rng.normal(size=(1, sys_.G, S))
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(struct.pack("3d", *cell) + struct.pack("3i", *ngrid) + struct.pack("i", len(sites)))
        for s in sites:
            f.write(struct.pack("3d", *s.R) + struct.pack("i", s.l) + struct.pack("2d", s.zeta, s.rc) +
                    struct.pack("i", s.species) +
                    struct.pack("d", s.zeta_dn if s.zeta_dn is not None else float("nan")))
        f.write(struct.pack("3d", *k) + struct.pack("i", S))
        f.write(np.ascontiguousarray(psi[0]).tobytes())
    r = subprocess.run([checker, str(inp), str(out)], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    J = sum(s.L for s in sites)
    dd = np.fromfile(out, dtype=np.complex128)
    spin = any(s.zeta_dn is not None for s in sites)
    dd = dd.reshape((2 if spin else 1), J, 3, S)
    e = SG.state_gradient_projections(sys_, psi, P.all_spheres(sys_))[0]
    assert normwise(dd[0], -e) < 1e-13
    if spin:
        # the spin-down table: the same sum over the spin-down orbitals
        dn = System(cell=cell, ngrid=ngrid, kpts=np.array([k]), kweights=np.ones(1), spin="unpolarized",
                    sites=[Site(R=s.R, l=s.l, zeta=(s.zeta_dn if s.zeta_dn is not None else s.zeta), rc=s.rc,
                                species=s.species) for s in sites])
        e_dn = SG.state_gradient_projections(dn, psi, P.all_spheres(dn))[0]
        assert normwise(dd[1], -e_dn) < 1e-13
