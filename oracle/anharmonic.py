"""Anharmonic stage of the oracle: three-phonon projections, scattering rates and
linewidths.  Plain FP64 NumPy; the projections phi+ and phi- are evaluated
separately and literally, for every (k, k') pair, as three successive tensor
contractions of the dense (mass-scaled, phased) third-order tensor.

Paper passages followed:
* Sec. II.B, eq. bose_einstein: n = 1 / (exp(hbar omega / k_B T) - 1).
* Sec. II.D, eq. Classic_n: classical occupation n = k_B T / (hbar omega).
* Sec. II.B, eq. projection_plus: phi+- = sum phi''' / sqrt(m m' m'')
  eta_ks eta+-_k's' eta*_k''s'' chi+-_k'l' chi*_k''l'', with eta+ = eta, chi+ = chi,
  eta- = eta*, chi- = chi*, chi_kl = exp(-i q_k . R_l).
* Sec. II.B, eq. gamma_operators: Gamma+- = (hbar pi / 8) g+- / (omega omega' omega'') |phi+-|^2.
* Sec. II.B, eq. phase_space: g+ = (n' - n'') delta+, g- = (1 + n' + n'') delta-,
  and the normalised phase space per mode g_mu that follows it.
* Sec. II.B, eq. delta_deconstructed: momentum Kronecker q +- q' - q'' = Q, and an
  energy delta.  The momentum delta is exact here: k'' = (k +- k') mod grid.
* Appendix A: the energy delta is a broadened function; the paper names three
  implementations, Gaussian, Lorentzian and triangular.
* Sec. II.B: Gamma^0 = sum (Gamma+ + Gamma-); tau = 1 / (2 Gamma^0).

Readings of points the paper leaves open:
* Normalisation of Gamma^0.  The linearised collision term of Sec. II.B carries
  1/N_k and a factor 1/2 on the creation (minus) processes; the printed
  Gamma^0 omits both.  Here gamma_mu = Gamma^0_mu =
  (1/N_k) [ sum_{k's's''} Gamma+ + 1/2 sum_{k's's''} Gamma- ], which is the
  Fermi-golden-rule half width (in rad/ps) of a phonon for the Hamiltonian
  term (1/3!) phi''' u u u of eq. potential_expansion.  The tests pin it
  against a Fock-space golden-rule calculation.
* The deltas are in angular frequency with width s = 2 pi sigma_THz and unit
  area, none truncated: Gaussian exp(-x^2 / 2 s^2) / (sqrt(2 pi) s) with s the
  standard deviation; Lorentzian s / (pi (x^2 + s^2)) with s the half width at
  half maximum; triangle max(0, 1 - |x| / s) / s with s the half base.  The
  paper gives no formula for the last two; these are their plain forms.
* Masked modes (nu < 0.01 THz) take no part as mu, mu' or mu''; their gamma is 0.
* Phase space per mode.  The paper normalises g_mu = sum_{mu' mu''} g / N
  without saying which N or how the two processes combine.  Here
  g_mu = (1/N_k) [ sum_{k's's''} g+ + 1/2 sum_{k's's''} g- ] in ps/rad: gamma_mu
  with the matrix-element factor (hbar pi / 8) |phi|^2 / (omega omega'
  omega'') replaced by 1, so the same counting (1/N_k, the 1/2 on creation).
* gamma is averaged over each degenerate set at k (only set averages are
  basis independent).
* Adaptive width (Appendix A: in crystals the width can be estimated from the
  phonon velocities; the paper cites that estimate and gives no formula).  For
  a process whose partners are q' and q'' (q'' fixed by momentum), the energy
  mismatch f(q') varies across one cell of the q grid with gradient
  v' - v'' (absorption) or v'' - v' (decay, q'' = q - q'); to first order a
  uniform q' over the cell, whose sides are b_a / G_a, spreads f with
  standard deviation sigma_grid = sqrt(sum_a ((v' - v'') . b_a / G_a)^2 / 12)
  (a uniform variable on an interval of width w has variance w^2 / 12).  The
  Gaussian of that process has standard deviation
  max(a sigma_grid, sigma_min), with a the user's scale and sigma_min the
  fixed width as a floor (v' = v'' would give a zero width).  Within a
  degenerate set a single mode's velocity depends on the eigenvector basis;
  the velocity used is the set mean (its trace), which does not.
"""

from __future__ import annotations

import numpy as np

from . import units
from .phonons import k_integer, k_index


def occupation(omega, T, stats='quantum'):
    """Equilibrium occupation at temperature T [K] for omega [rad/ps]."""
    omega = np.asarray(omega, dtype=float)
    with np.errstate(divide='ignore', over='ignore', invalid='ignore'):
        if stats == 'classical':
            return units.KB * T / (units.HBAR * omega)
        if T == 0:
            return np.zeros_like(omega)
        x = units.HBAR * omega / (units.KB * T)
        return 1.0 / np.expm1(x)


def gaussian_delta(x, sigma_omega):
    return np.exp(-0.5 * (x / sigma_omega) ** 2) / (np.sqrt(2.0 * np.pi) * sigma_omega)


def lorentzian_delta(x, sigma_omega):
    """Lorentzian of half width at half maximum sigma_omega, unit area."""
    return sigma_omega / (np.pi * (x * x + sigma_omega * sigma_omega))


def triangular_delta(x, sigma_omega):
    """Triangle of half base sigma_omega (zero beyond), unit area."""
    return np.maximum(0.0, 1.0 - np.abs(x) / sigma_omega) / sigma_omega


DELTAS = {'gauss': gaussian_delta, 'lorentz': lorentzian_delta, 'triangle': triangular_delta}


def adaptive_velocity_projections(crystal, ph):
    """U[k, s, a] = vbar_ks . b_a / G_a [rad/ps]: the degenerate-set mean group
    velocity of each mode projected on the reciprocal vectors b_a (rows of
    2 pi cell^-T) over the grid divisions G_a (Appendix A, adaptive width)."""
    b = 2.0 * np.pi * np.linalg.inv(crystal.cell).T           # rows: reciprocal vectors [rad/A]
    G = np.asarray(ph.grid, dtype=float)
    vbar = ph.velocity.copy()
    for k in range(ph.n_k):
        for S in ph.sets[k]:
            vbar[k, S] = vbar[k, S].mean(axis=0)
    return np.einsum('ksx,ax->ksa', vbar, b) / G[None, None, :]


def adaptive_sigma(U1, U2, scale, sigma_min):
    """Gaussian standard deviation of processes whose two partner modes have
    projections U1 and U2 (broadcast, last axis a): max(scale sqrt(sum_a (U1 -
    U2)^2 / 12), sigma_min)."""
    d = U1 - U2
    return np.maximum(scale * np.sqrt(np.sum(d * d, axis=-1) / 12.0), sigma_min)


def rate_prefactor():
    """(hbar pi / 8) with |phi|^2 in eV^2/(A^6 amu^3), omega in rad/ps -> rad/ps."""
    return np.pi / 8.0 * units.HBAR * units.EV_IN_AMU_A2_PS2 ** 3


def partner_index(ph, k, sign):
    """k'' = (k + sign k') mod grid, for every k'."""
    g = ph.grid
    mk = k_integer(k, g)
    out = np.empty(ph.n_k, dtype=np.int64)
    for kp in range(ph.n_k):
        mp = k_integer(kp, g)
        out[kp] = k_index([mk[c] + sign * mp[c] for c in range(3)], g)
    return out


def _phased_tensor(crystal, ph, kps, kpps, sign):
    """F[k', a, a', a''] = sum_blocks phi / sqrt(m m' m'') chi+-_{k'}(R1) chi*_{k''}(R2)."""
    n = crystal.n_modes
    nkp = len(kps)
    qp = ph.q[kps]                      # (nkp, 3)
    qpp = ph.q[kpps]
    R1 = crystal.fc3_R1.astype(float)
    R2 = crystal.fc3_R2.astype(float)
    if sign > 0:
        chi_p = np.exp(-2j * np.pi * (qp @ R1.T))     # chi_{k' l'}
    else:
        chi_p = np.exp(+2j * np.pi * (qp @ R1.T))     # chi*_{k' l'}
    chi_pp = np.exp(+2j * np.pi * (qpp @ R2.T))       # chi*_{k'' l''}
    phase = chi_p * chi_pp                             # (nkp, nb)
    m = crystal.masses
    scale = 1.0 / np.sqrt(m[crystal.fc3_i] * m[crystal.fc3_j] * m[crystal.fc3_l])
    vals = (crystal.fc3_val * scale[:, None, None, None]).reshape(-1, 27)
    F = np.zeros((nkp, n, n, n), dtype=np.complex128)
    triples = {}
    for b, key in enumerate(zip(crystal.fc3_i, crystal.fc3_j, crystal.fc3_l)):
        triples.setdefault(key, []).append(b)
    for (i, j, l), blist in triples.items():
        blist = np.asarray(blist)
        S = phase[:, blist] @ vals[blist]              # (nkp, 27)
        F[:, 3 * i:3 * i + 3, 3 * j:3 * j + 3, 3 * l:3 * l + 3] += S.reshape(nkp, 3, 3, 3)
    return F


def projection(crystal, ph, k, sign, kps=None):
    """phi^{sign}_{(k,s),(k',s'),(k'',s'')} for the listed k' (default: all).

    Returns (V[k', s, s', s''], k''[k'])."""
    if kps is None:
        kps = np.arange(ph.n_k)
    kps = np.asarray(kps)
    kpp_all = partner_index(ph, k, sign)
    kpps = kpp_all[kps]
    F = _phased_tensor(crystal, ph, kps, kpps, sign)
    Ek = ph.eigvec[k]
    Ep = ph.eigvec[kps] if sign > 0 else ph.eigvec[kps].conj()
    Epp = ph.eigvec[kpps].conj()
    # the three contractions (over a, then a', then a''), each as a (batched) matmul
    nkp, n = F.shape[0], F.shape[1]
    X = np.tensordot(F, Ek, axes=([1], [0]))                       # [k', a', a'', s]
    Y = np.matmul(np.swapaxes(Ep, 1, 2), X.reshape(nkp, n, n * n))  # [k', s', (a'', s)]
    Y = Y.reshape(nkp, n, n, n).transpose(0, 1, 3, 2)               # [k', s', s, a'']
    V = np.matmul(Y.reshape(nkp, n * n, n), Epp)                   # [k', (s', s), s'']
    V = V.reshape(nkp, n, n, n).transpose(0, 2, 1, 3)               # [k', s, s', s'']
    return V, kpps


def _set_average(ph, k, g):
    out = g.copy()
    for S in ph.sets[k]:
        out[..., S] = np.mean(g[..., S], axis=-1, keepdims=True)
    return out


def linewidths(crystal, ph, T, sigma_thz, stats='quantum', k_subset=None, average=True, delta='gauss',
               adaptive=None):
    """gamma_mu [rad/ps] for every mode mu = (k, s), k in k_subset, each T.

    ``delta`` picks the finite-width energy delta of the appendix (Gaussian,
    Lorentzian or triangular; width 2 pi sigma_thz in angular frequency).
    ``adaptive`` (a scale a, Gaussian only, needs ph with velocities): each
    process gets its own width max(a sigma_grid, 2 pi sigma_thz) from the
    velocities of its two partner modes (see the module header).
    Returns an array (nT, len(k_subset), n)."""
    delta_fn = DELTAS[delta]
    if adaptive is not None:
        assert delta == 'gauss'
        U = adaptive_velocity_projections(crystal, ph)
    T = np.atleast_1d(np.asarray(T, dtype=float))
    ks = np.arange(ph.n_k) if k_subset is None else np.asarray(k_subset)
    n = crystal.n_modes
    sig = units.TWO_PI * sigma_thz
    pref = rate_prefactor()
    out = np.zeros((len(T), len(ks), n))
    # partners k' are processed in chunks that bound the dense tensor to ~256 MB
    chunk = max(1, int(2 ** 28 // (16 * n ** 3)))
    for ik, k in enumerate(ks):
        w = ph.omega[k]
        mk = ph.mask[k]
        acc = np.zeros((len(T), n))
        for sign in (+1, -1):
          for c0 in range(0, ph.n_k, chunk):
            kps = np.arange(c0, min(ph.n_k, c0 + chunk))
            V, kpps = projection(crystal, ph, k, sign, kps=kps)
            V2 = np.abs(V) ** 2                                 # (k' chunk, s, s', s'')
            w1 = w[None, :, None, None]
            w2 = ph.omega[kps][:, None, :, None]
            w3 = ph.omega[kpps][:, None, None, :]
            m3 = (mk[None, :, None, None] & ph.mask[kps][:, None, :, None]
                  & ph.mask[kpps][:, None, None, :])
            with np.errstate(divide='ignore', invalid='ignore'):
                inv = np.where(m3, 1.0 / (w1 * w2 * w3), 0.0)
            if adaptive is None:
                delta = delta_fn(w1 + sign * w2 - w3, sig)
            else:
                s_e = adaptive_sigma(U[kps][:, None, :, None, :], U[kpps][:, None, None, :, :], adaptive, sig)
                delta = delta_fn(w1 + sign * w2 - w3, s_e)
            for it, t in enumerate(T):
                n2 = np.where(ph.mask[kps][:, None, :, None], occupation(w2, t, stats), 0.0)
                n3 = np.where(ph.mask[kpps][:, None, None, :], occupation(w3, t, stats), 0.0)
                if sign > 0:
                    g = (n2 - n3) * delta
                    G = pref * g * inv * V2
                    acc[it] += np.sum(G, axis=(0, 2, 3))
                else:
                    g = (1.0 + n2 + n3) * delta
                    G = pref * g * inv * V2
                    acc[it] += 0.5 * np.sum(G, axis=(0, 2, 3))
        acc /= ph.n_k
        acc[:, ~mk] = 0.0
        out[:, ik] = _set_average(ph, k, acc) if average else acc
    return out


def phase_space(ph, T, sigma_thz, stats='quantum', k_subset=None, delta='gauss'):
    """Normalised three-phonon phase space per mode g_mu [ps/rad] (Sec. II.B,
    eq. phase_space and the per-mode sum that follows it), every T.

    g_mu = (1/N_k) [ sum_{k's's''} (n' - n'') delta(w + w' - w'')
                     + 1/2 sum_{k's's''} (1 + n' + n'') delta(w - w' - w'') ]
    with k'' = k + k' (plus) and k'' = k - k' (minus).  Depends on frequencies
    only, so degenerate modes agree without averaging.  Returns (nT, len(k_subset), n)."""
    delta_fn = DELTAS[delta]
    T = np.atleast_1d(np.asarray(T, dtype=float))
    ks = np.arange(ph.n_k) if k_subset is None else np.asarray(k_subset)
    n = ph.omega.shape[1]
    sig = units.TWO_PI * sigma_thz
    out = np.zeros((len(T), len(ks), n))
    for ik, k in enumerate(ks):
        w = ph.omega[k]
        mk = ph.mask[k]
        acc = np.zeros((len(T), n))
        for sign in (+1, -1):
            kpps = partner_index(ph, k, sign)
            w1 = w[None, :, None, None]
            w2 = ph.omega[:, None, :, None]
            w3 = ph.omega[kpps][:, None, None, :]
            m3 = mk[None, :, None, None] & ph.mask[:, None, :, None] & ph.mask[kpps][:, None, None, :]
            d = np.where(m3, delta_fn(w1 + sign * w2 - w3, sig), 0.0)
            for it, t in enumerate(T):
                n2 = np.where(ph.mask[:, None, :, None], occupation(w2, t, stats), 0.0)
                n3 = np.where(ph.mask[kpps][:, None, None, :], occupation(w3, t, stats), 0.0)
                if sign > 0:
                    acc[it] += np.sum((n2 - n3) * d, axis=(0, 2, 3))
                else:
                    acc[it] += 0.5 * np.sum((1.0 + n2 + n3) * d, axis=(0, 2, 3))
        acc /= ph.n_k
        acc[:, ~mk] = 0.0
        out[:, ik] = acc
    return out


def linewidths_gamma_sparse(crystal, ph, T, sigma_thz, stats='quantum', s_subset=None, delta='gauss'):
    """Gamma-point-only linewidths for large cells, per first mode s.

    Same definitions as ``linewidths`` with N_k = 1 (all phases are 1); the
    third-order tensor is contracted with eta_s first into a sparse n x n
    matrix, then with the other two eigenvector sets.  No set averaging
    (returns raw per-mode values; disordered cells have no degeneracies above
    the acoustic modes)."""
    assert ph.n_k == 1
    delta_kind = delta
    T = np.atleast_1d(np.asarray(T, dtype=float))
    n = crystal.n_modes
    E = ph.eigvec[0]
    if not np.any(E.imag):
        # real eigenvectors at Gamma: same numbers, real arithmetic (contiguous for BLAS)
        E = np.ascontiguousarray(E.real)
    w = ph.omega[0]
    mask = ph.mask[0]
    sig = units.TWO_PI * sigma_thz
    pref = rate_prefactor()
    ss = np.arange(n) if s_subset is None else np.asarray(s_subset)
    m = crystal.masses
    scale = 1.0 / np.sqrt(m[crystal.fc3_i] * m[crystal.fc3_j] * m[crystal.fc3_l])
    vals = crystal.fc3_val * scale[:, None, None, None]     # (nb, 3,3,3)
    rows = (3 * crystal.fc3_j[:, None, None] + np.arange(3)[None, :, None]).repeat(3, axis=2)
    cols = (3 * crystal.fc3_l[:, None, None] + np.arange(3)[None, None, :]).repeat(3, axis=1)
    out = np.zeros((len(T), len(ss)))
    for idx, s in enumerate(ss):
        if not mask[s]:
            continue
        ea = E[3 * crystal.fc3_i[:, None] + np.arange(3)[None, :], s]        # (nb, 3)
        contrib = np.einsum('bx,bxyz->byz', ea, vals)                          # (nb, 3, 3)
        F = np.zeros((n, n), dtype=contrib.dtype)
        np.add.at(F, (rows.ravel(), cols.ravel()), contrib.ravel())
        w2 = w[:, None]
        w3 = w[None, :]
        m2 = mask[:, None] & mask[None, :]
        with np.errstate(divide='ignore', invalid='ignore'):
            inv = np.where(m2, 1.0 / (w[s] * w2 * w3), 0.0)
        acc = np.zeros(len(T))
        for sign in (+1, -1):
            Ep = E if sign > 0 else E.conj()
            V = Ep.T @ F @ E.conj()                       # V[s', s'']
            V2 = np.abs(V) ** 2
            delta = DELTAS[delta_kind](w[s] + sign * w2 - w3, sig)
            for it, t in enumerate(T):
                n2 = np.where(mask, occupation(w, t, stats), 0.0)[:, None]
                n3 = np.where(mask, occupation(w, t, stats), 0.0)[None, :]
                if sign > 0:
                    acc[it] += np.sum(pref * (n2 - n3) * delta * inv * V2)
                else:
                    acc[it] += 0.5 * np.sum(pref * (1.0 + n2 + n3) * delta * inv * V2)
        out[:, idx] = acc
    return out
