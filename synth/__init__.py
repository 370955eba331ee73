"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds no arithmetic of the Hubbard method: it only draws geometry
(cell, grid, atom positions, shell parameters, k-points) and Kohn-Sham-like
states (random sums of periodic Gaussians, orthonormalized on the grid) with
occupations.  Both the HIP path and the oracle receive exactly these arrays.
"""

from .configs import Config, make_config, CONFIG_NAMES  # noqa: F401
from .states import make_states, make_occupations  # noqa: F401
