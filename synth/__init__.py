"""Seeded synthetic inputs for the symmetry-blocked BSE hot path.

This module draws random numbers and shapes them into the inputs of the
Tamm-Dancoff two-particle Hamiltonian (band energies, mixed-basis pair vectors,
Coulomb and screened interactions, dipoles).  It holds none of the method's
arithmetic: every table that says which k points or k pairs share data
(orbit representatives, swap classes, the group action) is computed by the
caller and passed in, so that the CPU oracle and the GPU library each feed it
their own tables.
"""
from .gen import (  # noqa: F401
    splitmix64, keyed_uniform, keyed_normal, keyed_complex,
    CONFIGS, config, batch_configs, band_energies, coulomb_diag, exchange_vectors,
    pair_vectors, screened_w, dipoles, omega_grid_from_range, ETA, NOMEGA,
)
