"""Pins of the oracle's harmonic stage against results fixed independently of
its own formulas: a closed-form optical frequency, real-space supercell
eigenvalues, Hermiticity / time reversal / acoustic sum rule, and finite
differences of omega(q)."""

import numpy as np
import pytest

from gen import diamond_si, random_crystal
from gen.crystals import KEATING_ALPHA, KEATING_BETA, M_SI, M_GE
from oracle import phonons as P
from tests.supercell import fold, dense_fc2

EV = 1.602176634e-19 / (1.66053906660e-27 * 1e-20 / 1e-24)   # eV -> amu A^2 / ps^2


@pytest.mark.parametrize("masses", [(M_SI, M_SI), (M_SI, M_GE)])
def test_keating_optical_gamma_closed_form(masses):
    # Keating zincblende/diamond: omega_TO(Gamma)^2 = 4 (alpha + beta) (1/m1 + 1/m2).
    c = diamond_si(grid=(1, 1, 1), masses=masses)
    w, _ = P.eigenmodes(c, np.zeros(3))
    expect = np.sqrt(4.0 * (KEATING_ALPHA + KEATING_BETA) * (1 / masses[0] + 1 / masses[1]) * EV)
    assert np.allclose(w[3:], expect, rtol=1e-12)
    assert np.all(np.abs(w[:3]) < 1e-5)


@pytest.mark.parametrize("grid", [(3, 2, 2), (2, 2, 2)])
def test_bloch_spectrum_equals_supercell_spectrum(grid):
    c = diamond_si(grid=grid, masses=(M_SI, M_GE))
    ph = P.phonons(c, velocities=False)
    sc = fold(c)
    H = dense_fc2(sc)
    m = np.repeat(sc.masses, 3)
    lam = np.linalg.eigvalsh(H / np.sqrt(np.outer(m, m)) * EV)
    lam_bloch = np.sort((np.sign(ph.omega) * ph.omega ** 2).ravel())
    assert np.allclose(np.sort(lam), lam_bloch, atol=1e-8 * lam.max())


def test_dynamical_matrix_hermitian_time_reversal_asr():
    rng = np.random.default_rng(5)
    c = random_crystal(5, 3, rng)
    for q in [np.array([0.1, 0.37, -0.2]), np.array([0.5, 0.0, 0.25])]:
        D = P.dynamical_matrix(c, q)
        assert np.allclose(D, D.conj().T, atol=1e-12 * np.abs(D).max())
        assert np.allclose(P.dynamical_matrix(c, -q), D.conj(), atol=1e-12 * np.abs(D).max())
    w, vec = P.eigenmodes(c, np.zeros(3))
    assert np.sum(np.abs(w) < 1e-4 * np.abs(w).max()) == 3
    # acoustic eigenvectors at Gamma are mass-weighted rigid translations
    m = np.repeat(c.masses, 3)
    T = np.zeros((c.n_modes, 3))
    for a in range(3):
        T[a::3, a] = np.sqrt(c.masses)
    T /= np.linalg.norm(T, axis=0)
    acoustic = vec[:, np.argsort(np.abs(w))[:3]]
    overlap = np.linalg.svd(T.T @ acoustic.real, compute_uv=False)
    assert np.allclose(overlap, 1.0, atol=1e-8)
    del m


def _fd_velocity(c, q_red, h=1e-5):
    """d omega / d q_cart by central differences of the eigenvalues."""
    out = np.zeros((c.n_modes, 3))
    for a in range(3):
        dq = np.zeros(3)
        dq[a] = h
        dred = c.cell @ dq / (2 * np.pi)      # Cartesian step -> reduced step
        wp, _ = P.eigenmodes(c, q_red + dred)
        wm, _ = P.eigenmodes(c, q_red - dred)
        out[:, a] = (wp - wm) / (2 * h)
    return out


@pytest.mark.parametrize("q", [(0.13, 0.27, 0.41), (0.31, -0.12, 0.05)])
def test_velocity_matches_finite_difference(q):
    rng = np.random.default_rng(11)
    for c in [diamond_si(masses=(M_SI, M_GE)), random_crystal(4, 3, rng)]:
        q = np.asarray(q)
        w, vec, v, W = P.mode_velocities(c, q)
        fd = _fd_velocity(c, q)
        gaps = np.diff(w)
        nondeg = np.ones(len(w), bool)
        nondeg[:-1] &= gaps > 1e-3
        nondeg[1:] &= gaps > 1e-3
        assert nondeg.sum() >= 3
        assert np.allclose(v[nondeg], fd[nondeg], rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def test_set_velocity_products_basis_invariant():
    # Gamma-X line point of diamond: doubly degenerate transverse branches.
    c = diamond_si()
    q = np.array([0.0, 0.25, 0.25])
    w, vec, v, W = P.mode_velocities(c, q)
    sets = P.degenerate_sets(w / (2 * np.pi))
    assert any(len(S) > 1 for S in sets)
    vv = P.set_velocity_products(w, W, sets)
    rng = np.random.default_rng(0)
    U = np.eye(len(w), dtype=complex)
    for S in sets:
        Z = rng.normal(size=(len(S), len(S))) + 1j * rng.normal(size=(len(S), len(S)))
        Q, _ = np.linalg.qr(Z)
        U[np.ix_(S, S)] = Q
    W2 = P.velocity_matrices(c, q, vec @ U)
    vv2 = P.set_velocity_products(w, W2, sets)
    assert np.allclose(vv, vv2, atol=1e-10 * np.abs(vv).max())
    # non-degenerate modes: set product reduces to v v^T
    for S in sets:
        if len(S) == 1:
            s = S[0]
            assert np.allclose(vv[s], np.outer(v[s], v[s]), atol=1e-10 * np.abs(vv).max())
