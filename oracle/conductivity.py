"""Conductivity stage of the oracle: modal heat capacity, RTA conductivity and
QHGK conductivity.  Plain FP64 NumPy.

Paper passages followed:
* Sec. II.B, eq. heat_capacity: c_mu = hbar omega_mu dn_mu/dT.
* Sec. II.B, eq. RTA: kappa = 1/(N_k V) sum_mu c_mu v_mu,a v_mu,b tau_mu,
  tau_mu = 1/(2 Gamma^0_mu).
* Sec. II.C, eq. conductivity_amorphous: kappa = (1/V) sum_{mu mu'} c_{mu mu'}
  v_{mu mu' a} v_{mu mu' b} tau_{mu mu'}.
* Sec. II.C, eq. twod_heat_capacity, generalized_velocity, lorentzian_amorphous.
* Sec. II.D: classical limit, c = c_{mu mu'} = k_B.
* Sec. II.C, eq. diffusivity_per_mode: D_mu = sum_mu' v_{mu mu'} tau_{mu mu'} v_{mu mu'}.

Readings of points the paper leaves open:
* The printed generalised heat capacity (hbar w w'/T)(n - n')/(w - w') is
  negative for w != w'; the sign is fixed to (hbar w w'/T)(n' - n)/(w - w'),
  which is positive, tends to c_mu as w' -> w and equals k_B in the classical
  limit.  When |w - w'| < 1e-9 w the limit c_mu at the mean frequency is used.
* The generalised velocity sums over the fc2 blocks (i, j, R) with the
  displacement x_i - (x_j + R) of the actual image, and D = phi''/sqrt(m m').
* V is the unit-cell volume and N_k the grid size for RTA; for QHGK (Gamma
  point) V is the cell volume and N_k = 1.
* Conductivity is in W/(m K); masked modes (nu < 0.01 THz) are excluded.
* The diffusivity is given per Cartesian direction a (|v_{mu mu' a}|^2), in
  mm^2/s, without the printed 1/(N_k V), which does not give a diffusivity's
  units; with c = k_B it satisfies k_B sum_mu D_mu,a = V kappa_aa.
* The QHGK bandwidth option (Appendix A) replaces every mode's linewidth in the
  Lorentzian lifetime by the one given width eta [rad/ps]: tau_{mu mu'} =
  2 eta / ((w - w')^2 + 4 eta^2), a Lorentzian in w - w' of half width 2 eta
  and area pi, the broadened delta of the Allen-Feldman model.
* The QHGK energy threshold (Appendix A) is read as keeping the pairs that
  are close in frequency: tau_{mu mu'} = 0 when |w - w'| > w_thr (the
  printed inequality, which would drop the diagonal, is reversed).
"""

from __future__ import annotations

import numpy as np

from . import units
from .anharmonic import occupation


def heat_capacity(omega, T, stats='quantum'):
    """c = hbar omega dn/dT [eV/K] (quantum) or k_B (classical)."""
    omega = np.asarray(omega, dtype=float)
    if stats == 'classical':
        return np.full_like(omega, units.KB)
    x = units.HBAR * omega / (units.KB * T)
    with np.errstate(over='ignore', invalid='ignore', divide='ignore'):
        h = 0.5 * x / np.sinh(0.5 * x)
        return units.KB * np.where(x == 0, 1.0, h * h)


def volume(crystal):
    return abs(np.linalg.det(crystal.cell))


def kappa_rta(crystal, ph, gamma, T, stats='quantum'):
    """gamma: (nT, Nk, n) set-averaged linewidths [rad/ps]. Returns (nT, 3, 3) W/m/K."""
    T = np.atleast_1d(np.asarray(T, dtype=float))
    V = volume(crystal)
    out = np.zeros((len(T), 3, 3))
    for it, t in enumerate(T):
        c = heat_capacity(ph.omega, t, stats)
        with np.errstate(divide='ignore', invalid='ignore'):
            tau = np.where(ph.mask, 1.0 / (2.0 * gamma[it]), 0.0)
        w = np.where(ph.mask, c * tau, 0.0)
        out[it] = np.einsum('ks,ksab->ab', w, ph.vv) / (ph.n_k * V)
    return out * units.KAPPA_TO_SI


def generalized_velocity(crystal, ph):
    """v_{mu mu' a} at Gamma, shape (3, n, n) in A/ps."""
    n = crystal.n_modes
    E = ph.eigvec[0]
    w = ph.omega[0]
    m = crystal.masses
    M = np.zeros((3, n, n))
    for i, j, R, b in zip(crystal.fc2_i, crystal.fc2_j, crystal.fc2_R, crystal.fc2_val):
        dx = crystal.positions[i] - (crystal.positions[j] + np.asarray(R, float) @ crystal.cell)
        blk = b / np.sqrt(m[i] * m[j]) * units.EV_IN_AMU_A2_PS2
        for a in range(3):
            M[a, 3 * i:3 * i + 3, 3 * j:3 * j + 3] += dx[a] * blk
    v = np.einsum('as,xab,bt->xst', E.conj(), M, E, optimize=True)
    with np.errstate(divide='ignore', invalid='ignore'):
        sq = np.sqrt(np.outer(np.abs(w), np.abs(w)))
        v = v / (2.0 * sq[None])
    mm = np.outer(ph.mask[0], ph.mask[0])
    return np.where(mm[None], v, 0.0)


def generalized_heat_capacity(omega, T, stats='quantum'):
    w1 = omega[:, None]
    w2 = omega[None, :]
    if stats == 'classical':
        return np.full((len(omega), len(omega)), units.KB)
    n = occupation(omega, T, stats)
    n1 = n[:, None]
    n2 = n[None, :]
    with np.errstate(divide='ignore', invalid='ignore'):
        c = units.HBAR * w1 * w2 / T * (n2 - n1) / (w1 - w2)
    near = np.abs(w1 - w2) < 1e-9 * np.maximum(np.abs(w1), np.abs(w2))
    cd = heat_capacity(0.5 * (w1 + w2), T, stats)
    return np.where(near, cd, c)


def lorentzian_lifetime(omega, gamma, bandwidth=None, threshold=None):
    """tau_{mu mu'} = (g + g') / ((w - w')^2 + (g + g')^2) (Sec. II.C, eq.
    lorentzian_amorphous) [ps]; with a bandwidth eta every g is eta; with a
    threshold, 0 where |w - w'| > threshold (Appendix A)."""
    if bandwidth is not None:
        gamma = np.full_like(np.asarray(omega, dtype=float), float(bandwidth))
    g = gamma[:, None] + gamma[None, :]
    dw = omega[:, None] - omega[None, :]
    with np.errstate(divide='ignore', invalid='ignore'):
        tau = g / (dw * dw + g * g)
    if threshold is not None:
        tau = np.where(np.abs(dw) > threshold, 0.0, tau)
    return tau


def mode_diffusivity(crystal, ph, gamma, bandwidth=None, threshold=None):
    """Mode diffusivity at Gamma (Sec. II.C, eq. diffusivity_per_mode), per
    Cartesian direction: D[t][mu][a] = sum_mu' |v_{mu mu' a}|^2 tau_{mu mu'}
    in mm^2/s, with tau the Lorentzian lifetime of the QHGK conductivity at
    the linewidths gamma[t].  The printed prefactor 1/(N_k V) would leave a
    diffusivity in the wrong units; it is read as the normalisation of the
    conductivity sum, not of D, and dropped.  gamma: (nT, 1, n) [rad/ps].
    Masked modes have D = 0 (their velocities are zero).  Within a degenerate
    set only the sum over the set is independent of the eigenvector basis, so
    D is averaged over each set, as the linewidths are.  bandwidth and
    threshold are the QHGK options of lorentzian_lifetime."""
    assert ph.n_k == 1
    v = generalized_velocity(crystal, ph)              # (3, n, n), A/ps
    w = ph.omega[0]
    n = len(w)
    out = np.zeros((gamma.shape[0], n, 3))
    for it in range(gamma.shape[0]):
        tau = lorentzian_lifetime(w, gamma[it, 0], bandwidth, threshold)     # ps
        for a in range(3):
            out[it, :, a] = np.sum(np.where(np.abs(v[a]) > 0, np.abs(v[a]) ** 2 * tau, 0.0), axis=1)
        for S in ph.sets[0]:
            out[it, S, :] = out[it, S, :].mean(axis=0)
    return out * 1e-2                                   # A^2/ps -> mm^2/s


def kappa_qhgk(crystal, ph, gamma, T, stats='quantum', bandwidth=None, threshold=None):
    """gamma: (nT, 1, n) linewidths at Gamma [rad/ps]. Returns (nT, 3, 3) W/m/K.
    bandwidth and threshold are the QHGK options of lorentzian_lifetime."""
    assert ph.n_k == 1
    T = np.atleast_1d(np.asarray(T, dtype=float))
    V = volume(crystal)
    v = generalized_velocity(crystal, ph)              # (3, n, n)
    w = ph.omega[0]
    mask = ph.mask[0]
    mm = np.outer(mask, mask)
    out = np.zeros((len(T), 3, 3))
    for it, t in enumerate(T):
        c = generalized_heat_capacity(w, t, stats)
        tau = lorentzian_lifetime(w, gamma[it, 0], bandwidth, threshold)
        wgt = np.where(mm, c * tau, 0.0)
        out[it] = np.real(np.einsum('st,ast,bst->ab', wgt, v, v.conj())) / V
    return out * units.KAPPA_TO_SI
