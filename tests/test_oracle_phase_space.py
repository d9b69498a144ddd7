"""Pins of the oracle's normalised phase space per mode (Sec. II.B, eq.
phase_space and the per-mode sum after eq. delta_deconstructed):

* a brute-force sum over every ordered triple of modes on the grid, with
  momentum conservation tested on the q vectors themselves (q +- q' - q'' a
  reciprocal lattice vector) instead of the oracle's partner indices;
* the closed form for a Lorentzian much wider than the spectrum, where the
  delta is the constant 1 / (pi s) and the sums reduce to per-k sums of
  occupations and mode counts (fixes the 1/N_k, the 1/2 on decay and the sign
  of n' - n'');
* classical statistics make g affine in T;
* modes of one degenerate set share g, masked modes have g = 0.
"""

import numpy as np
import pytest

from gen import diamond_si
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A

TWO_PI = 2.0 * np.pi


@pytest.fixture(scope="module")
def diamond_232():
    c = diamond_si(grid=(2, 3, 2), rc3=2.6, masses=(M_SI, M_GE), seed=8)
    return c, P.phonons(c, velocities=False)


def _partners(q):
    """plus[k, k'] = k'' with q_k + q_k' - q_k'' integer; minus[k, k'] with q_k - q_k' - q_k''."""
    nk = len(q)
    plus = np.full((nk, nk), -1)
    minus = np.full((nk, nk), -1)
    for k in range(nk):
        for kp in range(nk):
            for kpp in range(nk):
                dp = q[k] + q[kp] - q[kpp]
                dm = q[k] - q[kp] - q[kpp]
                if np.allclose(dp, np.round(dp), atol=1e-9):
                    plus[k, kp] = kpp
                if np.allclose(dm, np.round(dm), atol=1e-9):
                    minus[k, kp] = kpp
    assert np.all(plus >= 0) and np.all(minus >= 0)
    return plus, minus


@pytest.mark.parametrize("delta,stats,T", [("gauss", "quantum", [0.0, 300.0]),
                                            ("lorentz", "classical", [300.0]),
                                            ("triangle", "quantum", [500.0])])
def test_brute_force_triples(diamond_232, delta, stats, T):
    c, ph = diamond_232
    sigma = 0.4
    s = TWO_PI * sigma
    g = A.phase_space(ph, T, sigma, stats=stats, delta=delta)
    nk, n = ph.omega.shape
    # every mode (k, s) as one flat list; all ordered triples
    w = ph.omega.reshape(-1)
    on = ph.mask.reshape(-1)
    kof = np.repeat(np.arange(nk), n)
    plus, minus = _partners(ph.q)
    delta_fn = A.DELTAS[delta]
    for it, t in enumerate(T):
        occ = np.where(on, A.occupation(w, t, stats), 0.0)
        ref = np.zeros(nk * n)
        for a in range(nk * n):
            if not on[a]:
                continue
            for b in range(nk * n):
                if not on[b]:
                    continue
                kb = kof[b]
                # third modes at the partner point of each process, all branches
                cp = plus[kof[a], kb] * n + np.arange(n)
                cm = minus[kof[a], kb] * n + np.arange(n)
                mp, mm = on[cp], on[cm]
                ref[a] += np.sum(mp * (occ[b] - occ[cp]) * delta_fn(w[a] + w[b] - w[cp], s))
                ref[a] += 0.5 * np.sum(mm * (1.0 + occ[b] + occ[cm]) * delta_fn(w[a] - w[b] - w[cm], s))
        ref /= nk
        assert np.allclose(g[it].reshape(-1), ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())
    if stats == "quantum" and T[0] == 0.0:
        assert np.all(g[0] >= 0.0)


def test_wide_lorentzian_closed_form(diamond_232):
    """With s much larger than every frequency, delta = 1/(pi s) (1 + O(x^2/s^2)):
    g_k = 1/(pi s N_k) sum_k' [ A(k') B(k+k') - B(k') A(k+k')
                               + 1/2 (B(k') B(k-k') + A(k') B(k-k') + B(k') A(k-k')) ]
    with B(k) the number of unmasked modes at k and A(k) their summed occupations."""
    c, ph = diamond_232
    s = 1e7                                   # rad/ps
    sigma = s / TWO_PI
    T = 250.0
    g = A.phase_space(ph, [T], sigma, delta="lorentz")[0]
    nk, n = ph.omega.shape
    occ = np.where(ph.mask, A.occupation(ph.omega, T), 0.0)
    Acnt = occ.sum(axis=1)
    Bcnt = ph.mask.sum(axis=1).astype(float)
    plus, minus = _partners(ph.q)
    for k in range(nk):
        tot = 0.0
        for kp in range(nk):
            a, b = plus[k, kp], minus[k, kp]
            tot += Acnt[kp] * Bcnt[a] - Bcnt[kp] * Acnt[a]
            tot += 0.5 * (Bcnt[kp] * Bcnt[b] + Acnt[kp] * Bcnt[b] + Bcnt[kp] * Acnt[b])
        ref = tot / (np.pi * s * nk)
        for j in range(n):
            if ph.mask[k, j]:
                assert g[k, j] == pytest.approx(ref, rel=1e-9)
            else:
                assert g[k, j] == 0.0


def test_classical_affine_in_temperature(diamond_232):
    c, ph = diamond_232
    T1, T2 = 200.0, 450.0
    g = A.phase_space(ph, [T1, T2, 2 * T2 - T1], 0.3, stats="classical")
    assert np.allclose(g[2], 2 * g[1] - g[0], rtol=1e-10, atol=1e-14 * np.abs(g).max())


def test_degenerate_sets_and_masked_modes(diamond_232):
    c, ph = diamond_232
    g = A.phase_space(ph, [300.0], 0.2)[0]
    for k in range(ph.n_k):
        for S in ph.sets[k]:
            if ph.mask[k, S[0]]:
                assert np.allclose(g[k, S], g[k, S[0]], rtol=1e-8)
    assert np.all(g[~ph.mask] == 0.0)
    assert np.all(g[ph.mask] > 0.0)
