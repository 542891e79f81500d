"""Seeded synthetic inputs for the LSMS tau00 path.

This package prepares what the path takes as input: fcc NiAu-shaped
supercells (positions, species, vacancies, positional noise), the list of
(site, energy) instances with their LIZ cutoff radii, the complex energy
contour (nodes and quadrature weights) and the square-well phase shifts that stand in for real muffin-tin
potentials (spin-split wells and canted moment directions for the
spin-canted case).  It contains no step of the path itself (no LIZ extraction, no
t-matrix, no structure constants, no factorisation); both the product path
and the oracle take their inputs from here.  The learned form's initial
network parameters are seeded inputs too (`mlp_init`).
"""

from .workloads import (  # noqa: F401
    A_LAT,
    MLP_LAYERS,
    R_MT,
    SPLIT_SPECIES,
    V0_SPECIES,
    Workload,
    canted_moments,
    config1,
    config2,
    config3,
    config4,
    config_canted,
    config_large,
    config_large_canted,
    contour_energies,
    contour_ends,
    contour_weights,
    fcc_supercell,
    mlp_init,
    phase_shift_table,
    spin_phase_shift_tables,
    square_well_delta,
    subset,
)
