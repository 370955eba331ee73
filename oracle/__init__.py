"""FP64 CPU oracle for the DFT+U / ACBN0 Hubbard kernel.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised numpy/scipy implementation of what the Hubbard hot path computes,
written from Tancogne-Dejean, Oliveira & Rubio, "Self-consistent DFT+U method
for real-space time-dependent density functional theory calculations"
(arXiv 1711.08935).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_1711_08935_amd``) never imports, links or executes anything here,
and nothing here imports the product path: the two share no code.

Everything is FP64 (complex128 where the states are complex).  Units are
Hartree atomic units.

Modules (each function cites the passage it follows):

* ``harmonics``   real spherical/solid harmonics (from scipy's complex Y_lm)
* ``orbitals``    localized orbitals on spheres, Bloch sums over images
                  (Sec. II, Fig. 1 and the sphere discussion that follows it)
* ``projection``  <phi_{I,m,k}|psi> by brute force over the whole cell grid
* ``occupations`` n (Eq. occ_matrices), N-bar and P-bar (Eqs. notation_Nbar,
                  notation_Pbar), spinor forms (App. A, App. B)
* ``coulomb``     on-site Coulomb tensor (mm'|m''m''') on the grid (Sec. III,
                  App. B notation), Hockney FFT and O(N^2) double sum;
                  continuum Slater-integral reference
* ``acbn0``       U-bar, J-bar (Eqs. ACBN0_U, ACBN0_J; App. B)
* ``potential``   V_U|psi> (Eq. pot_V_U), Dudarev E_U (Eq. E_Dudarev and its
                  noncollinear form in App. A)
* ``forces``      Hubbard forces (Sec. IV) and finite-difference checks
* ``step``        one whole Hubbard step from the functions above
* ``gauge``       velocity-gauge projection and apply, the DFT+U current
                  correction (Sec. V)
* ``fll``         noncollinear HF energy and FLL double counting with the
                  magnetization of the shell (App. A)
* ``spinorb``     spin-dependent orbitals of noncollinear runs (App. A)
* ``radius``      sphere radius selection (Sec. II, radius discussion)
* ``stencil``     forces through <phi|grad psi> with a 4th-order central
                  difference of the states (Sec. IV, the paper's own form)

Parity pins live in ``tests/test_oracle_*.py``.  A function whose values no
independent property fixes would say "parity unpinned" in its module
header; none does.
"""

from . import harmonics, orbitals, projection, occupations, coulomb, acbn0, potential, forces, step, gauge, stencil, radius, fll, spinorb  # noqa: F401
from .orbitals import System, Site  # noqa: F401
