"""Plain FP64 CPU oracle for the three-phonon linewidth path (test infrastructure).

This package is test infrastructure only.  It is imported by the tests, by the
smoke check and by the CPU-baseline leg of the benchmark, and by nothing else:
the GPU library never calls it, and it shares no code, constants or tables with
the GPU library.

It evaluates the definitions of Barbalinardo et al., "Efficient Anharmonic
Lattice Dynamics Calculations of Thermal Transport in Crystalline and
Disordered Solids" (arXiv:2009.01967) literally, in float64, with NumPy/LAPACK:

* ``phonons``      -- dynamical matrix, Bloch transform and eigenmodes
                      (Sec. II.A, eq. eigenvectors / eigenvectors_crystal),
                      group velocities (Sec. II.B, eq. velocity_crystal).
* ``anharmonic``   -- Bose-Einstein occupations (eq. bose_einstein), the
                      projections phi+ and phi- (eq. projection_plus), phase-space
                      weights and scattering rates (eq. gamma_operators,
                      phase_space, delta_deconstructed), and the linewidth
                      Gamma^0 (Sec. II.B).
* ``conductivity`` -- modal heat capacity (eq. heat_capacity), RTA conductivity
                      (eq. RTA), and the QHGK conductivity with generalised heat
                      capacity, velocity and Lorentzian lifetime (Sec. II.C,
                      eqs. conductivity_amorphous .. lorentzian_amorphous), and
                      the classical limit (Sec. II.D).

* ``scattering``   -- the full linearised BTE: the off-diagonal operator
                      Gamma^1 (Sec. II.B), the conductivity by direct inversion
                      (eqs. inversemeanfreepath, full_conductivity) and by the
                      self-consistent series (eqs. mfp_from_scattering_inv,
                      self-consistent).
* ``interpolation`` -- linewidths interpolated in frequency with a natural
                      cubic spline, from a smaller cell to a larger one (Sec.
                      II.C, Sec. IV.B).

Readings of points the paper leaves open are listed in each module's header.
Every function here is pinned by tests that do not re-type its formula.
"""

from . import units, phonons, anharmonic, conductivity, scattering, interpolation  # noqa: F401
