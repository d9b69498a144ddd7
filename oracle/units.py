"""Physical constants for the oracle (CODATA 2018), in the oracle's unit system.

Length Angstrom, mass amu, energy eV, time ps, temperature K.
Angular frequencies are in rad/ps; frequencies nu = omega / 2 pi are in THz.
"""

import math

HBAR = 6.582119569e-4          # eV ps
KB = 8.617333262e-5            # eV / K
EV = 1.602176634e-19           # J
AMU = 1.66053906660e-27        # kg

# 1 eV expressed in amu A^2 / ps^2.
EV_IN_AMU_A2_PS2 = EV / (AMU * 1e-20 / 1e-24)

# eV / (K A ps) -> W / (m K):  J / (K m s).
KAPPA_TO_SI = EV / (1e-10 * 1e-12)

TWO_PI = 2.0 * math.pi

# Modes with nu below this (THz) are excluded everywhere (zero / imaginary).
NU_MIN_THZ = 0.01
# Two modes at the same k belong to one degenerate set when their frequencies
# differ by less than this (THz), chained over the sorted spectrum.
DEGENERACY_THZ = 1e-5
