"""Pins of the oracle's adaptive delta width (Appendix A: the width estimated
from the phonon velocities): the width is the spread of the energy mismatch
over one cell of the q grid, checked by sampling that cell and evaluating the
frequencies there; it halves when the grid doubles; a zero scale gives the
fixed width exactly; and the linewidths do not depend on the eigenvector basis
inside degenerate sets (the set-mean velocity enters)."""

import numpy as np
import pytest

from gen import diamond_si, random_crystal
from oracle import phonons as P, anharmonic as A


def _nondegenerate(ph, k):
    return [S[0] for S in ph.sets[k] if len(S) == 1 and ph.mask[k, S[0]]]


def test_adaptive_width_is_the_spread_of_the_mismatch_over_a_grid_cell():
    """Absorption q + q' -> q'': move q' (and with it q'' = q + q') uniformly
    over a cell, t_a in [-1/2, 1/2] along lam b_a / G_a; the standard
    deviation of w + w'(q') - w''(q'') is lam sqrt(sum_a ((v' - v'') .
    b_a / G_a)^2 / 12) to first order.  A quarter of the grid cell (lam =
    1/4) keeps the curvature of the bands out of the comparison."""
    c = random_crystal(3, 24, np.random.default_rng(11))
    G = np.asarray(c.grid, dtype=float)
    ph = P.phonons(c)
    U = A.adaptive_velocity_projections(c, ph)
    rng = np.random.default_rng(2)
    checked = 0
    for k, kp in ((5, 130), (777, 4321), (2000, 9000)):
        kpp = A.partner_index(ph, k, +1)[kp]
        s1s, s2s = _nondegenerate(ph, kp), _nondegenerate(ph, kpp)
        lam = 0.25
        t = lam * rng.uniform(-0.5, 0.5, size=(4000, 3)) / G     # reduced offsets within the cell
        w1 = np.array([P.eigenmodes(c, ph.q[kp] + d)[0] for d in t])
        w2 = np.array([P.eigenmodes(c, ph.q[kpp] + d)[0] for d in t])
        for s1, s2 in ((s1s[0], s2s[-1]), (s1s[len(s1s) // 2], s2s[len(s2s) // 2])):
            f = w1[:, s1] - w2[:, s2]
            sigma = A.adaptive_sigma(U[kp, s1], U[kpp, s2], 1.0, 0.0)
            assert sigma > 0.05
            assert np.std(f) / lam == pytest.approx(sigma, rel=0.03), (k, kp, s1, s2)
            checked += 1
    assert checked == 6


def test_adaptive_width_halves_when_the_grid_doubles():
    c4 = diamond_si(grid=(4, 4, 4), rc3=2.6)
    c8 = diamond_si(grid=(8, 8, 8), rc3=2.6)
    ph4, ph8 = P.phonons(c4), P.phonons(c8)
    U4, U8 = A.adaptive_velocity_projections(c4, ph4), A.adaptive_velocity_projections(c8, ph8)
    for k4 in range(ph4.n_k):
        m = P.k_integer(k4, (4, 4, 4))
        k8 = P.k_index([2 * x for x in m], (8, 8, 8))
        assert np.allclose(ph8.omega[k8], ph4.omega[k4], rtol=1e-12, atol=1e-9)
        assert np.allclose(U8[k8], 0.5 * U4[k4], rtol=1e-9, atol=1e-9)


def test_zero_scale_gives_the_fixed_width():
    c = diamond_si(grid=(3, 3, 3), rc3=2.6)
    ph = P.phonons(c)
    g0 = A.linewidths(c, ph, [300.0], 0.3, k_subset=[0, 4])
    ga = A.linewidths(c, ph, [300.0], 0.3, k_subset=[0, 4], adaptive=0.0)
    assert np.array_equal(g0, ga)
    gb = A.linewidths(c, ph, [300.0], 0.3, k_subset=[0, 4], adaptive=1.0)
    assert not np.allclose(g0, gb, rtol=1e-3)


def test_adaptive_linewidths_do_not_depend_on_the_basis_of_degenerate_sets():
    """A random unitary inside every degenerate set, with the velocities
    recomputed from the rotated eigenvectors, leaves gamma unchanged."""
    c = diamond_si(grid=(3, 3, 3), rc3=2.6)
    ph = P.phonons(c)
    rng = np.random.default_rng(9)
    E = ph.eigvec.copy()
    vel = ph.velocity.copy()
    rotated = 0
    for k in range(ph.n_k):
        for S in ph.sets[k]:
            if len(S) > 1:
                Z = rng.normal(size=(len(S), len(S))) + 1j * rng.normal(size=(len(S), len(S)))
                Q, _ = np.linalg.qr(Z)
                E[k][:, S] = E[k][:, S] @ Q
                rotated += 1
        W = P.velocity_matrices(c, ph.q[k], E[k])
        with np.errstate(divide='ignore', invalid='ignore'):
            vel[k] = np.where(ph.mask[k][:, None], np.real(np.einsum('xss->sx', W)) / (2.0 * ph.omega[k][:, None]),
                              0.0)
    assert rotated > 10
    ph2 = P.Phonons(grid=ph.grid, q=ph.q, omega=ph.omega, eigvec=E, mask=ph.mask, sets=ph.sets,
                    velocity=vel, vv=ph.vv)
    assert not np.allclose(vel, ph.velocity, atol=1e-3)
    ks = [1, 13]
    g1 = A.linewidths(c, ph, [300.0], 0.1, k_subset=ks, adaptive=1.0)
    g2 = A.linewidths(c, ph2, [300.0], 0.1, k_subset=ks, adaptive=1.0)
    assert np.allclose(g1, g2, rtol=1e-10, atol=1e-14)
