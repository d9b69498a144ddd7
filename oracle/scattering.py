"""Full linearised BTE stage of the oracle: the off-diagonal scattering operator,
the conductivity by direct inversion and by the self-consistent series.
Plain FP64 NumPy/LAPACK, test infrastructure only.

Paper passages followed (Sec. II.B):
* the linearised scattering term of the BTE (the expression with psi_mu,
  psi_mu', psi_mu'' before eq. gamma_operators), which fixes how each
  three-phonon rate couples the deviations of its three modes;
* v_mu = sum_mu' (delta_mu mu' Gamma^0_mu + Gamma^1_mu mu') lambda_mu', with
  Gamma^1_mu mu' = (w_mu' / w_mu) sum_mu'' (Gamma+_mu mu' mu'' - Gamma+_mu mu'' mu'
  - Gamma-_mu mu' mu'' - Gamma-_mu mu'' mu');
* eq. inversemeanfreepath and eq. full_conductivity: lambda = Gamma~^-1 v and
  kappa = 1/(N_k V) sum c_mu v_mu Gamma~^-1_mu mu' v_mu';
* eq. mfp_from_scattering_inv and eq. self-consistent: the geometric series
  lambda = sum_n (-Gamma^1 / Gamma^0)^n lambda^0.

Readings of points the paper leaves open:
* Normalisation of Gamma^1.  The scattering term carries 1/N_k and a factor
  1/2 on the creation rates; the printed Gamma^0 and Gamma^1 omit both.  As for
  Gamma^0 (the linewidth), both are kept here:
    Gamma^1_mu nu = (w_nu / w_mu) (1/N_k) sum_mu'' [ Gamma+_mu nu mu''
                    - Gamma+_mu mu'' nu - 1/2 Gamma-_mu nu mu'' - 1/2 Gamma-_mu mu'' nu ],
  which is exactly the coefficient of psi_nu in the scattering term when the
  coefficient of psi_mu is Gamma^0_mu (pinned against that term summed
  triple by triple).
* Factor 2.  With Gamma^1 = 0, eq. full_conductivity must give the RTA
  conductivity of eq. RTA, whose lifetime is tau = 1/(2 Gamma^0); the inverse
  is therefore taken of 2 (Gamma^0 + Gamma^1): Gamma^0 is the half width, the
  relaxation rate of the population is twice that.  The self-consistent
  series starts from lambda^0 = v / (2 Gamma^0), and the factor cancels in its
  recursion.
* Degenerate modes.  Inside a set of degenerate modes the per-mode rates
  depend on the eigenvector basis; only sums over the set do not.  As gamma is
  averaged over each set, the operator is averaged over each pair of sets:
  on the vectors that are constant within every set it is the block sum
  sum_{a in A, b in B} Gamma^1_ab / sqrt(|A| |B|) (orthonormal set vectors),
  and it is zero on the vectors that sum to zero within a set, which thus
  relax with the set-averaged Gamma^0 alone (RTA).  The velocity then enters
  through basis invariants: the set mean m_A = Tr(W) / (2 w |A|) and the set
  sum of v v (Re Tr(W_a W_b) / (4 w^2), as in the RTA conductivity).
* Time reversal.  The velocity is odd under k -> -k and the operator commutes
  with that map, so the mean free path is odd too: both methods work on the
  odd set vectors (e_A - e_A') / sqrt(2), A' the set of -k that mirrors set A
  of k.  This is exact, halves the system, and leaves out the even vectors,
  among them the uniform deviation that energy conservation makes a (near)
  zero mode of the operator; on them the series of eq. mfp_from_scattering_inv
  can diverge even when it converges on the odd vectors.  Sets at points with
  k = -k (mod the grid) have no odd vector; their velocity vanishes and they
  keep only the within-set (RTA) part.
* Masked modes (nu < 0.01 THz) take no part.
"""

from __future__ import annotations

import numpy as np

from . import units
from .anharmonic import DELTAS, occupation, projection, rate_prefactor
from .conductivity import heat_capacity, volume


def scattering_operator(crystal, ph, T, sigma_thz, stats='quantum', delta='gauss'):
    """Gamma^0 (per mode, not set averaged) and Gamma^1 (per mode pair) in
    rad/ps for every temperature.  Modes are numbered mu = k n + s.

    Returns (G0 [nT][Nk n], G1 [nT][Nk n][Nk n])."""
    delta_fn = DELTAS[delta]
    T = np.atleast_1d(np.asarray(T, dtype=float))
    nk, n = ph.n_k, crystal.n_modes
    nm = nk * n
    sig = units.TWO_PI * sigma_thz
    pref = rate_prefactor()
    G0 = np.zeros((len(T), nm))
    X = np.zeros((len(T), nm, nm))      # the bracket of Gamma^1, before 1/N_k and w_nu / w_mu
    chunk = max(1, int(2 ** 28 // (16 * n ** 3)))
    for k in range(nk):
        w = ph.omega[k]
        mk = ph.mask[k]
        rows = k * n + np.arange(n)
        for sign in (+1, -1):
            for c0 in range(0, nk, chunk):
                kps = np.arange(c0, min(nk, c0 + chunk))
                V, kpps = projection(crystal, ph, k, sign, kps=kps)      # V[k', s, s', s'']
                V2 = np.abs(V) ** 2
                w1 = w[None, :, None, None]
                w2 = ph.omega[kps][:, None, :, None]
                w3 = ph.omega[kpps][:, None, None, :]
                m3 = (mk[None, :, None, None] & ph.mask[kps][:, None, :, None]
                      & ph.mask[kpps][:, None, None, :])
                with np.errstate(divide='ignore', invalid='ignore'):
                    inv = np.where(m3, 1.0 / (w1 * w2 * w3), 0.0)
                dl = delta_fn(w1 + sign * w2 - w3, sig)
                for it, t in enumerate(T):
                    n2 = np.where(ph.mask[kps][:, None, :, None], occupation(w2, t, stats), 0.0)
                    n3 = np.where(ph.mask[kpps][:, None, None, :], occupation(w3, t, stats), 0.0)
                    if sign > 0:
                        G = pref * (n2 - n3) * dl * inv * V2             # Gamma+_{mu, mu', mu''}
                        G0[it, rows] += G.sum(axis=(0, 2, 3))
                        w_mid, w_last = +1.0, -1.0                       # + Gamma+_{mu nu .} - Gamma+_{mu . nu}
                    else:
                        G = pref * (1.0 + n2 + n3) * dl * inv * V2       # Gamma-_{mu, mu', mu''}
                        G0[it, rows] += 0.5 * G.sum(axis=(0, 2, 3))
                        w_mid, w_last = -0.5, -0.5                       # - 1/2 Gamma-_{mu nu .} - 1/2 Gamma-_{mu . nu}
                    # nu in the middle: nu = (k', s'), summed over s''
                    mid = G.sum(axis=3)                                   # [k', s, s']
                    for a, kp in enumerate(kps):
                        X[it, rows[:, None], kp * n + np.arange(n)[None, :]] += w_mid * mid[a]
                    # nu last: nu = (k'', s''), summed over s'
                    last = G.sum(axis=2)                                  # [k', s, s'']
                    for a, kpp in enumerate(kpps):
                        X[it, rows[:, None], kpp * n + np.arange(n)[None, :]] += w_last * last[a]
    G0 /= nk
    X /= nk
    om = ph.omega.reshape(-1)
    mask = ph.mask.reshape(-1)
    with np.errstate(divide='ignore', invalid='ignore'):
        ratio = np.where(mask[:, None] & mask[None, :], om[None, :] / om[:, None], 0.0)
    G0[:, ~mask] = 0.0
    return G0, X * ratio[None]


def mode_sets(ph):
    """Global degenerate sets of the unmasked modes (index arrays into
    mu = k n + s) and, per set, the index of its time-reversed set at -k."""
    from .phonons import k_integer, k_index
    n = ph.omega.shape[1]
    out, key = [], {}
    for k in range(ph.n_k):
        for Sx in ph.sets[k]:
            Sx = np.asarray(Sx)
            if ph.mask[k, Sx].all():
                key[(k, int(Sx[0]))] = len(out)
                out.append(k * n + Sx)
    tr = np.zeros(len(out), dtype=np.int64)
    for a, Sx in enumerate(out):
        k = int(Sx[0]) // n
        km = k_index([-x for x in k_integer(k, ph.grid)], ph.grid)
        tr[a] = key[(km, int(Sx[0]) % n)]
        assert len(out[tr[a]]) == len(Sx)
    return out, tr


def set_invariants(ph, sets):
    """Per set: size d, mean velocity m [3] (A/ps) and the set sum of v v [3][3]
    ((A/ps)^2, Re Tr(W_a W_b) / (4 w^2))."""
    vel = ph.velocity.reshape(-1, 3)
    vv = ph.vv.reshape(-1, 3, 3)
    d = np.array([len(S) for S in sets], dtype=float)
    m = np.array([vel[S].mean(axis=0) for S in sets])
    tv = np.array([vv[S].sum(axis=0) for S in sets])
    return d, m, tv


def reduce_to_sets(G0, G1, sets):
    """Set-averaged Gamma^0 [nS] and the operator on the set vectors
    B[A][B] = sum_{a in A, b in B} G1[a][b] / sqrt(|A| |B|)."""
    nS = len(sets)
    g0 = np.array([G0[S].mean() for S in sets])
    B = np.zeros((nS, nS))
    for ia, SA in enumerate(sets):
        rowsum = G1[SA].sum(axis=0)
        for ib, SB in enumerate(sets):
            B[ia, ib] = rowsum[SB].sum() / np.sqrt(len(SA) * len(SB))
    return g0, B


def odd_reduce(g0, B, u, tr):
    """The problem on the odd set vectors o_i = (e_a - e_a') / sqrt(2), one per
    pair a < a' = tr[a]: representatives a, g0 [r], B_odd [r][r], u_odd [r][3]."""
    reps = np.array([a for a in range(len(tr)) if a < tr[a]], dtype=np.int64)
    ta = tr[reps]
    Bo = 0.5 * (B[np.ix_(reps, reps)] - B[np.ix_(reps, ta)] - B[np.ix_(ta, reps)] + B[np.ix_(ta, ta)])
    uo = (u[reps] - u[ta]) / np.sqrt(2.0)
    return reps, g0[reps], Bo, uo


def kappa_from_operator(c, d, m, tv, g0, B, tr, V, nk, method='inverse', max_iter=500, tol=1e-14):
    """kappa [3][3] in W/(m K) of the set-reduced problem, and (terms, converged)
    of the self-consistent series (None for the inverse).

    c, d, g0: per set heat capacity [eV/K], size and set-averaged Gamma^0;
    m, tv: mean velocity and set sum of v v; B: the off-diagonal operator on
    the set vectors; tr: the time-reversed set of each set.  The within-set
    deviations of v relax with Gamma^0 alone; the set means solve
    2 (diag(g0) + B) L = sqrt(d) m on the odd set vectors, by direct
    inversion or by the series."""
    u = np.sqrt(d)[:, None] * m                                  # components of v on the set vectors
    reps, go, Bo, uo = odd_reduce(g0, B, u, tr)
    info = None
    if method == 'inverse':
        L = np.linalg.solve(2.0 * (np.diag(go) + Bo), uo)
    else:
        L, nit, ok = self_consistent_mean(go, Bo, uo, max_iter, tol)
        info = (nit, ok)
    dev = tv - d[:, None, None] * m[:, :, None] * m[:, None, :]
    k = np.einsum('a,abc->bc', c / (2.0 * g0), dev) + np.einsum('a,ab,ac->bc', c[reps], uo, L)
    return k / (nk * V) * units.KAPPA_TO_SI, info


def self_consistent_mean(g0, B, u, max_iter=500, tol=1e-14):
    """Partial sums of eq. mfp_from_scattering_inv: L_0 = lambda^0 = u / (2 g0),
    then each step adds the next term lambda^{n+1} = -(1/Gamma^0) Gamma^1 lambda^n
    of eq. self-consistent.  Stops when the last term is below tol times the
    sum.  Returns (L, number of terms added, converged)."""
    lam0 = u / (2.0 * g0)[:, None]
    L = lam0.copy()
    term = lam0.copy()
    for it in range(1, max_iter + 1):
        term = -(B @ term) / g0[:, None]
        L = L + term
        if np.abs(term).max() <= tol * np.abs(L).max():
            return L, it, True
    return L, max_iter, False


def kappa_bte(crystal, ph, T, sigma_thz, stats='quantum', delta='gauss', method='inverse',
              offdiagonal=True, max_iter=500, tol=1e-14):
    """Conductivity of the full linearised BTE, (nT, 3, 3) W/(m K).

    method 'inverse' (eq. full_conductivity) or 'self-consistent' (eq.
    self-consistent, summed until converged).  offdiagonal=False drops
    Gamma^1 (the RTA).  For 'self-consistent' also returns, per temperature,
    the number of terms and whether the series converged."""
    T = np.atleast_1d(np.asarray(T, dtype=float))
    G0, G1 = scattering_operator(crystal, ph, T, sigma_thz, stats, delta)
    sets, tr = mode_sets(ph)
    d, m, tv = set_invariants(ph, sets)
    om = ph.omega.reshape(-1)
    Vc = volume(crystal)
    out = np.zeros((len(T), 3, 3))
    infos = []
    for it, t in enumerate(T):
        g0, B = reduce_to_sets(G0[it], G1[it], sets)
        if not offdiagonal:
            B = np.zeros_like(B)
        # heat capacity averaged over each set, like gamma (the set's modes
        # differ by less than the degeneracy threshold)
        cm = heat_capacity(om, t, stats)
        c = np.array([cm[S].mean() for S in sets])
        out[it], info = kappa_from_operator(c, d, m, tv, g0, B, tr, Vc, ph.n_k, method, max_iter, tol)
        infos.append(info)
    return (out, infos) if method != 'inverse' else out
