"""Harmonic stage of the oracle: dynamical matrix, Bloch transform, eigenmodes,
group velocities.  Plain FP64 NumPy/LAPACK, no blocking or reordering.

Paper passages followed:
* Sec. II.A, after eq. second_and_third_ifc: D = phi'' / sqrt(m m').
* Sec. II.A, eq. eigenvectors / eigenvectors_crystal: D(q_k) = sum_l chi_kl D(0, l)
  with chi_kl = exp(-i q_k . R_l), eigenpairs D(q_k) eta_ks = omega_ks^2 eta_ks.
* Sec. II.B, eq. velocity_crystal: v = d omega / d q by Hellmann-Feynman.

Readings of points the paper leaves open:
* The q grid is Gamma centred and unshifted, q_k = (m1/G1, m2/G2, m3/G3) in
  reduced reciprocal coordinates, k = (m1 G2 + m2) G3 + m3, so q +- q' stays on
  the grid.  The phase uses the lattice vector R_l only.
* omega = sign(lambda) sqrt(|lambda|); modes with nu < 0.01 THz (acoustic modes
  at Gamma, imaginary modes) are masked out everywhere.
* The printed velocity formula drops a conjugate and a primed index; the
  Hellmann-Feynman form used here is v_s = Re(eta_s^H dD/dq eta_s) / (2 omega_s)
  with dD/dq_alpha = sum_R (-i R_alpha) D_R exp(-i q.R).  Inside a degenerate set
  only basis-invariant quantities are meaningful; for the conductivity the set
  sum of v_alpha v_beta is Re Tr(W_alpha W_beta) / (4 omega^2) with
  W = E_set^H dD E_set.
* Degenerate sets: modes at one k whose sorted frequencies are chained by gaps
  below 1e-5 THz.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from . import units


def qpoints(grid) -> np.ndarray:
    """Reduced coordinates of the Gamma-centred grid, row k = (m1 G2 + m2) G3 + m3."""
    g = [int(x) for x in grid]
    m = np.array(np.meshgrid(np.arange(g[0]), np.arange(g[1]), np.arange(g[2]),
                             indexing='ij')).reshape(3, -1).T
    return m / np.asarray(g, dtype=float)


def k_index(m, grid) -> int:
    g = [int(x) for x in grid]
    return int(((m[0] % g[0]) * g[1] + (m[1] % g[1])) * g[2] + (m[2] % g[2]))


def k_integer(k, grid):
    g = [int(x) for x in grid]
    return (k // (g[1] * g[2]), (k // g[2]) % g[1], k % g[2])


def dynamical_matrix(crystal, q) -> np.ndarray:
    """D(q) in ps^-2: sum over fc2 blocks of phi/sqrt(m_i m_j) exp(-2 pi i q.R)."""
    n = crystal.n_modes
    D = np.zeros((n, n), dtype=np.complex128)
    m = crystal.masses
    for i, j, R, v in zip(crystal.fc2_i, crystal.fc2_j, crystal.fc2_R, crystal.fc2_val):
        chi = np.exp(-2j * np.pi * np.dot(q, R))
        D[3 * i:3 * i + 3, 3 * j:3 * j + 3] += chi * v / np.sqrt(m[i] * m[j])
    return D * units.EV_IN_AMU_A2_PS2


def dynamical_matrix_gradient(crystal, q) -> np.ndarray:
    """dD/dq_alpha (Cartesian q, 1/A) in ps^-2 A, shape (3, n, n)."""
    n = crystal.n_modes
    dD = np.zeros((3, n, n), dtype=np.complex128)
    m = crystal.masses
    for i, j, R, v in zip(crystal.fc2_i, crystal.fc2_j, crystal.fc2_R, crystal.fc2_val):
        chi = np.exp(-2j * np.pi * np.dot(q, R))
        Rc = np.asarray(R, dtype=float) @ crystal.cell
        for a in range(3):
            dD[a, 3 * i:3 * i + 3, 3 * j:3 * j + 3] += (-1j * Rc[a]) * chi * v / np.sqrt(m[i] * m[j])
    return dD * units.EV_IN_AMU_A2_PS2


def degenerate_sets(nu_sorted) -> List[np.ndarray]:
    sets = []
    cur = [0]
    for s in range(1, len(nu_sorted)):
        if abs(nu_sorted[s] - nu_sorted[s - 1]) < units.DEGENERACY_THZ:
            cur.append(s)
        else:
            sets.append(np.array(cur))
            cur = [s]
    sets.append(np.array(cur))
    return sets


@dataclass
class Phonons:
    grid: tuple
    q: np.ndarray            # (Nk, 3) reduced
    omega: np.ndarray        # (Nk, n) rad/ps, signed
    eigvec: np.ndarray       # (Nk, n, n) complex, column s = eta_ks
    mask: np.ndarray         # (Nk, n) bool, nu >= NU_MIN
    sets: list               # per k: list of index arrays
    velocity: np.ndarray     # (Nk, n, 3) A/ps, per-mode Hellmann-Feynman
    vv: np.ndarray           # (Nk, n, 3, 3): set trace Re Tr(W_a W_b)/(4 w^2) / |set|

    @property
    def nu(self):
        return self.omega / units.TWO_PI

    @property
    def n_k(self):
        return self.q.shape[0]


def eigenmodes(crystal, q):
    """omega [rad/ps] (ascending, signed) and eigenvectors (columns) of D(q)."""
    D = dynamical_matrix(crystal, q)
    D = 0.5 * (D + D.conj().T)
    if not np.any(q):
        # At Gamma D is real symmetric: keep real eigenvectors.
        lam, vec = np.linalg.eigh(D.real)
        vec = vec.astype(np.complex128)
    else:
        lam, vec = np.linalg.eigh(D)
    return np.sign(lam) * np.sqrt(np.abs(lam)), vec


def velocity_matrices(crystal, q, vec):
    """W_alpha = E^H dD/dq_alpha E, shape (3, n, n) [ps^-2 A]."""
    dD = dynamical_matrix_gradient(crystal, q)
    return np.einsum('as,xab,bt->xst', vec.conj(), dD, vec, optimize=True)


def mode_velocities(crystal, q):
    """(omega, eigvec, v[s, alpha] = Re W_alpha[s, s] / (2 omega_s), W)."""
    w, vec = eigenmodes(crystal, q)
    W = velocity_matrices(crystal, q, vec)
    with np.errstate(divide='ignore', invalid='ignore'):
        v = np.real(np.einsum('xss->sx', W)) / (2.0 * w[:, None])
    return w, vec, v, W


def set_velocity_products(w, W, sets):
    """Per mode: Re Tr(W_a W_b) / (4 omega^2) over its degenerate set, / |set|."""
    n = len(w)
    vv = np.zeros((n, 3, 3))
    for S in sets:
        Wa = W[:, S][:, :, S]                                 # (3, |S|, |S|)
        tr = np.real(np.einsum('ast,bts->ab', Wa, Wa))      # Tr(W_a W_b)
        wS = np.mean(w[S])
        with np.errstate(divide='ignore', invalid='ignore'):
            vv[S] = tr / (4.0 * wS * wS) / len(S)
    return vv


def phonons(crystal, grid=None, velocities=True) -> Phonons:
    grid = tuple(crystal.grid if grid is None else grid)
    q = qpoints(grid)
    nk, n = q.shape[0], crystal.n_modes
    omega = np.zeros((nk, n))
    E = np.zeros((nk, n, n), dtype=np.complex128)
    vel = np.zeros((nk, n, 3))
    vv = np.zeros((nk, n, 3, 3))
    sets = []
    for k in range(nk):
        if velocities:
            w, vec, v, W = mode_velocities(crystal, q[k])
        else:
            w, vec = eigenmodes(crystal, q[k])
        omega[k] = w
        E[k] = vec
        sk = degenerate_sets(w / units.TWO_PI)
        sets.append(sk)
        if velocities:
            vel[k] = v
            vv[k] = set_velocity_products(w, W, sk)
    mask = (omega / units.TWO_PI) >= units.NU_MIN_THZ
    vel[~mask] = 0.0
    vv[~mask] = 0.0
    return Phonons(grid=grid, q=q, omega=omega, eigvec=E, mask=mask, sets=sets,
                   velocity=vel, vv=vv)
