"""Pins of the oracle's full linearised BTE (Sec. II.B: the off-diagonal
operator Gamma^1, eq. inversemeanfreepath / full_conductivity and the
self-consistent series of eqs. mfp_from_scattering_inv / self-consistent):

* the operator (Gamma^0 on the diagonal plus Gamma^1) applied to a random
  deviation equals the paper's linearised scattering term summed triple by
  triple over all momentum-conserving (mu, mu', mu'') with the q vectors;
* without Gamma^1 the inversion gives the RTA conductivity of eq. RTA;
* a hand-built two-set problem solved in closed form;
* the self-consistent series converges to the direct inverse when the
  off-diagonal part is smaller than the diagonal on the odd vectors;
* the full set-space solve is odd under time reversal and agrees with the
  odd-vector solve;
* rotating the eigenvectors inside degenerate sets leaves kappa unchanged;
* kappa scales as 1/s^2 under fc3 -> s fc3."""

import numpy as np
import pytest

from gen import diamond_si
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A, conductivity as C, scattering as S, units

SIGMA = 0.25


@pytest.fixture(scope="module")
def small():
    """Two species, 3x3x3 grid (points off the time-reversal-invariant ones,
    so velocities are nonzero), first-shell fc3."""
    c = diamond_si(grid=(3, 3, 3), rc3=2.6, masses=(M_SI, M_GE), seed=21)
    return c, P.phonons(c)


def _q_in_lattice(q):
    return np.allclose(q, np.round(q), atol=1e-12)


def test_operator_equals_scattering_term_triple_by_triple(small):
    c, ph = small
    T = 300.0
    nk, n = ph.n_k, c.n_modes
    G0, G1 = S.scattering_operator(c, ph, [T], SIGMA)
    rng = np.random.default_rng(5)
    psi = rng.standard_normal(nk * n)
    lhs = G0[0] * psi + G1[0] @ psi
    # the linearised scattering term, one triple at a time
    w = ph.omega.reshape(-1)
    mask = ph.mask.reshape(-1)
    sig = units.TWO_PI * SIGMA
    pref = A.rate_prefactor()
    nocc = np.where(mask, A.occupation(w, T), 0.0)
    rhs = np.zeros(nk * n)
    for k in range(nk):
        for kp in range(nk):
            for sign in (+1, -1):
                V, kpp = A.projection(c, ph, k, sign, kps=[kp])
                kpp = int(kpp[0])
                assert _q_in_lattice(ph.q[k] + sign * ph.q[kp] - ph.q[kpp])
                for s in range(n):
                    mu = k * n + s
                    if not mask[mu]:
                        continue
                    for s1 in range(n):
                        m1 = kp * n + s1
                        for s2 in range(n):
                            m2 = kpp * n + s2
                            if not (mask[m1] and mask[m2]):
                                continue
                            x = w[mu] + sign * w[m1] - w[m2]
                            d = np.exp(-0.5 * (x / sig) ** 2) / (np.sqrt(2 * np.pi) * sig)
                            occ = (nocc[m1] - nocc[m2]) if sign > 0 else (1.0 + nocc[m1] + nocc[m2])
                            rate = pref * occ * d * abs(V[0, s, s1, s2]) ** 2 / (w[mu] * w[m1] * w[m2])
                            if sign > 0:
                                term = rate * (w[mu] * psi[mu] + w[m1] * psi[m1] - w[m2] * psi[m2])
                            else:
                                term = 0.5 * rate * (w[mu] * psi[mu] - w[m1] * psi[m1] - w[m2] * psi[m2])
                            rhs[mu] += term / (w[mu] * nk)
    scale = np.abs(rhs).max()
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-12 * scale)
    # the diagonal is the linewidth
    g = A.linewidths(c, ph, [T], SIGMA, average=False)[0].reshape(-1)
    assert np.allclose(G0[0], g, rtol=1e-12, atol=1e-14 * g.max())


def test_without_offdiagonal_is_rta(small):
    c, ph = small
    T = [150.0, 600.0]
    k_bte = S.kappa_bte(c, ph, T, SIGMA, offdiagonal=False)
    g = A.linewidths(c, ph, T, SIGMA)
    k_rta = C.kappa_rta(c, ph, g, T)
    assert np.allclose(k_bte, k_rta, rtol=1e-12, atol=1e-12 * np.abs(k_rta).max())


def test_hand_built_two_set_problem():
    """Four singleton sets, two pairs mirrored by time reversal (sets 0 <-> 2,
    1 <-> 3) with odd velocities v_x = (1, 0.5, -1, -0.5), gamma^0 =
    (1, 2, 1, 2), c = 1, V = N_k = 1.  Gamma^1 couples 0 -> 1 by 0.5 and
    1 -> 0 by 0.25 (and mirrored), nothing across the pairs, so on the odd
    vectors 2 (Gamma^0 + Gamma^1) = [[2, 1], [0.5, 4]] with right-hand side
    sqrt(2) (1, 0.5): the solution is sqrt(2) (3.5, 0.5) / 7.5 and
    kappa_xx = 2 (1 * 3.5 + 0.5 * 0.5) / 7.5 = 1."""
    d = np.ones(4)
    m = np.array([[1.0, 0, 0], [0.5, 0, 0], [-1.0, 0, 0], [-0.5, 0, 0]])
    tv = np.einsum('ab,ac->abc', m, m)
    g0 = np.array([1.0, 2.0, 1.0, 2.0])
    B = np.zeros((4, 4))
    B[0, 1] = B[2, 3] = 0.5
    B[1, 0] = B[3, 2] = 0.25
    tr = np.array([2, 3, 0, 1])
    c = np.ones(4)
    k, info = S.kappa_from_operator(c, d, m, tv, g0, B, tr, 1.0, 1)
    k = k / units.KAPPA_TO_SI
    assert info is None
    assert k[0, 0] == pytest.approx(1.0, rel=1e-15)
    assert np.abs(k.ravel()[1:]).max() == 0.0
    ks, (nit, ok) = S.kappa_from_operator(c, d, m, tv, g0, B, tr, 1.0, 1, method='self-consistent')
    assert ok and nit < 40
    assert ks[0, 0] / units.KAPPA_TO_SI == pytest.approx(1.0, rel=1e-13)


@pytest.fixture(scope="module")
def converging():
    """Two species on a 4x4x4 grid: on the odd vectors the off-diagonal part is
    smaller than the diagonal (spectral radius about 0.65 at 300 K)."""
    c = diamond_si(grid=(4, 4, 4), rc3=2.6, masses=(M_SI, M_GE), seed=21)
    return c, P.phonons(c)


def test_self_consistent_series_converges_to_inverse(converging):
    c, ph = converging
    T = [300.0]
    G0, G1 = S.scattering_operator(c, ph, T, SIGMA)
    sets, tr = S.mode_sets(ph)
    g0, B = S.reduce_to_sets(G0[0], G1[0], sets)
    d, m, _ = S.set_invariants(ph, sets)
    _, go, Bo, _ = S.odd_reduce(g0, B, np.sqrt(d)[:, None] * m, tr)
    rho = np.abs(np.linalg.eigvals(Bo / go[:, None])).max()
    assert rho < 1.0, rho
    k_inv = S.kappa_bte(c, ph, T, SIGMA, method='inverse')
    k_sc, info = S.kappa_bte(c, ph, T, SIGMA, method='self-consistent', tol=1e-15, max_iter=2000)
    assert info[0][1], info
    assert np.allclose(k_sc, k_inv, rtol=1e-11, atol=1e-12 * np.abs(k_inv).max())
    # a series stopped early is further away
    k_10, info10 = S.kappa_bte(c, ph, T, SIGMA, method='self-consistent', max_iter=10)
    assert not info10[0][1]
    assert np.abs(k_10 - k_inv).max() > 1e3 * np.abs(k_sc - k_inv).max()
    # the off-diagonal part moves kappa away from the RTA
    k_rta = S.kappa_bte(c, ph, T, SIGMA, offdiagonal=False)
    assert np.abs(k_inv - k_rta).max() > 1e-4 * np.abs(k_rta).max()


def test_odd_solution_equals_full_solution(small):
    """The mean free path of the whole set space, solved directly, is odd under
    time reversal and gives the same kappa as the odd-vector solve."""
    c, ph = small
    G0, G1 = S.scattering_operator(c, ph, [300.0], SIGMA)
    sets, tr = S.mode_sets(ph)
    g0, B = S.reduce_to_sets(G0[0], G1[0], sets)
    d, m, _ = S.set_invariants(ph, sets)
    u = np.sqrt(d)[:, None] * m
    L = np.linalg.solve(2.0 * (np.diag(g0) + B), u)
    assert np.allclose(L[tr], -L, rtol=1e-6, atol=1e-9 * np.abs(L).max())
    reps, go, Bo, uo = S.odd_reduce(g0, B, u, tr)
    Lo = np.linalg.solve(2.0 * (np.diag(go) + Bo), uo)
    assert np.allclose(Lo, (L[reps] - L[tr[reps]]) / np.sqrt(2.0), rtol=1e-6, atol=1e-9 * np.abs(Lo).max())


def test_kappa_independent_of_eigenvector_basis_in_degenerate_sets():
    """Pure-Si diamond has degenerate sets; a random unitary inside every set
    changes the per-mode rates but not kappa."""
    c = diamond_si(grid=(3, 3, 3), rc3=2.6, seed=22)
    ph = P.phonons(c)
    assert max(len(Sx) for sk in ph.sets for Sx in sk) > 1
    k0 = S.kappa_bte(c, ph, [300.0], SIGMA)
    rng = np.random.default_rng(8)
    E = ph.eigvec.copy()
    for k in range(ph.n_k):
        for Sx in ph.sets[k]:
            d = len(Sx)
            if d > 1:
                Z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
                U, _ = np.linalg.qr(Z)
                E[k][:, Sx] = E[k][:, Sx] @ U
    ph2 = P.Phonons(grid=ph.grid, q=ph.q, omega=ph.omega, eigvec=E, mask=ph.mask, sets=ph.sets,
                    velocity=ph.velocity, vv=ph.vv)
    k1 = S.kappa_bte(c, ph2, [300.0], SIGMA)
    assert np.allclose(k1, k0, rtol=1e-11, atol=1e-12 * np.abs(k0).max())


def test_kappa_scales_as_inverse_fc3_squared(small):
    c, ph = small
    k1 = S.kappa_bte(c, ph, [300.0], SIGMA)
    k2 = S.kappa_bte(c.with_fc3_scaled(2.0), ph, [300.0], SIGMA)
    assert np.allclose(4.0 * k2, k1, rtol=1e-12)
