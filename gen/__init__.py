"""Seeded synthetic crystals and glasses for the three-phonon linewidth path.

This package only *builds inputs*: lattice, positions, masses, second-order
force constants (fc2) and third-order force constants (fc3), all in the
home-cell-first block format that both the CPU oracle and the GPU library
consume.  It contains none of the linewidth or conductivity arithmetic.

Units: Angstrom, amu, eV (fc2 in eV/A^2, fc3 in eV/A^3).
"""

from .crystals import (  # noqa: F401
    Crystal,
    diamond_si,
    cage_cell,
    random_crystal,
    sige_supercell,
    batch_crystals,
    WORKLOADS,
    workload,
)
