"""Pins of the oracle's three-phonon projection and linewidths against results
fixed independently of its formulas:

* a Fock-space Fermi-golden-rule calculation (ladder-operator matrices) for a
  three-mode system, which fixes the hbar pi / 8 prefactor, the 1/2 on creation
  processes, the occupation factors, tau = 1/(2 gamma) and the unit chain;
* a brute-force real-space sum over the grid supercell, which fixes the Bloch
  phases, conjugations and momentum conservation of phi+ and phi-;
* permutation identities of |phi|, the acoustic sum rule at Gamma, exact
  scalings, time reversal, and the folded-supercell Gamma-point calculation that
  fixes the 1/N_k normalisation.
"""

import itertools

import numpy as np
import pytest

from gen import diamond_si, sige_supercell
from gen.crystals import Crystal, M_SI, M_GE
from oracle import phonons as P, anharmonic as A
from tests.supercell import fold, dense_fc3

# Constants typed independently of the oracle (CODATA 2018).
HBAR = 6.582119569e-4                                         # eV ps
KB = 8.617333262e-5                                           # eV/K
EV = 1.602176634e-19 / (1.66053906660e-27 * 1e-20 / 1e-24)   # eV -> amu A^2/ps^2


# ----------------------------------------------------------------------------
# Fock-space golden rule
# ----------------------------------------------------------------------------

def _molecule(freqs, m=28.09, seed=3, t_scale=4.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    w = np.asarray(freqs, float)
    K = m * Q @ np.diag(w ** 2) @ Q.T / EV                  # eV/A^2
    K = 0.5 * (K + K.T)
    T = rng.normal(size=(3, 3, 3)) * t_scale
    T = sum(np.transpose(T, p) for p in itertools.permutations(range(3))) / 6.0
    z = np.zeros((1, 3), np.int32)
    c = Crystal(name='three-mode', cell=np.eye(3) * 10.0, positions=np.zeros((1, 3)),
                masses=np.array([m]), fc2_i=np.array([0], np.int32), fc2_j=np.array([0], np.int32),
                fc2_R=z, fc2_val=K[None], fc3_i=np.array([0], np.int32),
                fc3_j=np.array([0], np.int32), fc3_l=np.array([0], np.int32), fc3_R1=z, fc3_R2=z,
                fc3_val=T[None], grid=(1, 1, 1))
    return c, Q, w, T, m


def _golden_rule_matrix_element(Q, w, T, m, initial, final, nmax=6):
    """<final| (1/3!) sum T u u u |initial> in eV with u_a = sum_s sqrt(hbar/2 m w_s) Q_as (b_s + b_s^+)."""
    d = nmax + 1
    b = np.diag(np.sqrt(np.arange(1, d)), 1)
    X = b + b.T
    I = np.eye(d)
    Xs = [np.kron(np.kron(X, I), I), np.kron(np.kron(I, X), I), np.kron(np.kron(I, I), X)]
    amp = np.sqrt(HBAR * EV / (2.0 * m * w))                 # A
    U = [sum(amp[s] * Q[a, s] * Xs[s] for s in range(3)) for a in range(3)]
    H3 = np.zeros((d ** 3, d ** 3))
    for a, b_, c in itertools.product(range(3), repeat=3):
        H3 += T[a, b_, c] * (U[a] @ U[b_] @ U[c])
    H3 /= 6.0

    def idx(o):
        return (o[0] * d + o[1]) * d + o[2]
    return H3[idx(final), idx(initial)]


def _gauss(x, s):
    return np.exp(-0.5 * (x / s) ** 2) / (np.sqrt(2 * np.pi) * s)


@pytest.mark.parametrize("T_K", [0.0, 300.0, 900.0])
def test_decay_rate_matches_fock_space_golden_rule(T_K):
    # mode 2 (10 rad/ps) decays into modes 0 and 1 (4.05 + 6 rad/ps)
    sig_thz = 0.02
    c, Q, w, T3, m = _molecule([4.05, 6.0, 10.0])
    ph = P.phonons(c, velocities=False)
    assert np.allclose(ph.omega[0], w, rtol=1e-10)
    # oracle eigenvectors may differ from Q by signs: the rate uses |M|^2 only
    M0 = _golden_rule_matrix_element(Q, w, T3, m, (0, 0, 1), (1, 1, 0))
    s = 2 * np.pi * sig_thz
    rate0 = 2 * np.pi * M0 ** 2 / HBAR ** 2 * _gauss(w[2] - w[0] - w[1], s)   # 1/ps at T = 0
    n = np.zeros(3) if T_K == 0 else 1.0 / np.expm1(HBAR * w / (KB * T_K))
    # relaxation rate of the population of mode 2: rate0 * [(1+n0)(1+n1) - n0 n1]
    rate = rate0 * ((1 + n[0]) * (1 + n[1]) - n[0] * n[1])
    gamma = A.linewidths(c, ph, [T_K], sig_thz)[0, 0]
    assert gamma[2] == pytest.approx(0.5 * rate, rel=1e-9)


@pytest.mark.parametrize("T_K", [150.0, 600.0])
def test_absorption_rate_matches_fock_space_golden_rule(T_K):
    # mode 0 (4.05) absorbs mode 1 (6) into mode 2 (10)
    sig_thz = 0.02
    c, Q, w, T3, m = _molecule([4.05, 6.0, 10.0], seed=8)
    ph = P.phonons(c, velocities=False)
    M0 = _golden_rule_matrix_element(Q, w, T3, m, (1, 1, 0), (0, 0, 1))
    # the same element with real occupations obeys bosonic enhancement
    M12 = _golden_rule_matrix_element(Q, w, T3, m, (1, 2, 1), (0, 1, 2))
    assert M12 ** 2 == pytest.approx(M0 ** 2 * 2 * 2, rel=1e-10)
    s = 2 * np.pi * sig_thz
    rate0 = 2 * np.pi * M0 ** 2 / HBAR ** 2 * _gauss(w[0] + w[1] - w[2], s)
    n = 1.0 / np.expm1(HBAR * w / (KB * T_K))
    # d n0/dt = -rate0 [n0 n1 (1 + n2) - (1 + n0)(1 + n1) n2]; linear coefficient in n0
    rate = rate0 * (n[1] * (1 + n[2]) - (1 + n[1]) * n[2])
    gamma = A.linewidths(c, ph, [T_K], sig_thz)[0, 0]
    assert gamma[0] == pytest.approx(0.5 * rate, rel=1e-9)
    gamma0 = A.linewidths(c, ph, [0.0], sig_thz)[0, 0]
    assert abs(gamma0[0]) < 1e-12 * abs(gamma[0])


@pytest.mark.parametrize("kind", ["gauss", "lorentz", "triangle"])
def test_delta_shapes_have_unit_area_and_their_stated_width(kind):
    from scipy.integrate import quad
    s = 0.7
    f = A.DELTAS[kind]
    if kind == "triangle":
        area = quad(lambda x: f(x, s), -s, s, points=[0.0])[0]
    else:
        area = quad(lambda x: f(x, s), -np.inf, np.inf)[0]
    assert area == pytest.approx(1.0, abs=1e-9)
    peak = f(0.0, s)
    if kind == "gauss":          # standard deviation s: second moment s^2
        m2 = quad(lambda x: x * x * f(x, s), -np.inf, np.inf)[0]
        assert m2 == pytest.approx(s * s, rel=1e-9)
    elif kind == "lorentz":      # half width at half maximum s
        assert f(s, s) == pytest.approx(0.5 * peak, rel=1e-12)
        assert f(-s, s) == pytest.approx(0.5 * peak, rel=1e-12)
    else:                        # half base s, linear flanks
        assert f(s, s) == 0.0 and f(1.5 * s, s) == 0.0
        assert f(0.5 * s, s) == pytest.approx(0.5 * peak, rel=1e-12)
    assert np.all(f(np.linspace(-5 * s, 5 * s, 101), s) >= 0.0)


@pytest.mark.parametrize("kind", ["lorentz", "triangle"])
def test_decay_rate_matches_golden_rule_with_each_delta(kind):
    # the Fock-space decay of mode 2 with the energy delta of the given kind, at
    # an exact resonance w2 = w0 + w1 and a width far below every other energy
    # mismatch, so that the Lorentzian tails of the other processes stay below
    # 1e-8 of the resonant term
    sig_thz, T_K = 1e-5, 300.0
    c, Q, w, T3, m = _molecule([4.05, 5.95, 10.0])
    ph = P.phonons(c, velocities=False)
    M0 = _golden_rule_matrix_element(Q, w, T3, m, (0, 0, 1), (1, 1, 0))
    s = 2 * np.pi * sig_thz
    wo = ph.omega[0]
    x = wo[2] - wo[0] - wo[1]
    d = s / (np.pi * (x * x + s * s)) if kind == "lorentz" else max(0.0, 1 - abs(x) / s) / s
    n = 1.0 / np.expm1(HBAR * w / (KB * T_K))
    rate = 2 * np.pi * M0 ** 2 / HBAR ** 2 * d * ((1 + n[0]) * (1 + n[1]) - n[0] * n[1])
    gamma = A.linewidths(c, ph, [T_K], sig_thz, delta=kind)[0, 0]
    assert gamma[2] == pytest.approx(0.5 * rate, rel=1e-7)


def test_deltas_agree_in_the_narrow_limit():
    # far from any resonance all three kinds vanish together; on the 2-atom
    # diamond the linewidth per kind converges as the width shrinks relative to
    # the spread of the energy mismatches
    c = diamond_si(grid=(3, 3, 3), rc3=2.6)
    ph = P.phonons(c, velocities=False)
    g = {k: A.linewidths(c, ph, [300.0], 0.05, delta=k) for k in ("gauss", "lorentz", "triangle")}
    for k in ("lorentz", "triangle"):
        assert np.all(np.isfinite(g[k])) and np.all(g[k] >= -1e-15)
    # identical support structure: where the Gaussian weight is exactly zero so is the triangle's
    assert np.all(g["triangle"][g["gauss"] == 0.0] == 0.0)


# ----------------------------------------------------------------------------
# Bloch conventions against real-space supercell sums
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def crystal_322():
    c = diamond_si(grid=(3, 2, 2), rc3=4.0, masses=(M_SI, M_GE), seed=77)
    ph = P.phonons(c, velocities=False)
    sc = fold(c)
    Tsc = dense_fc3(sc)
    msc = np.repeat(sc.masses, 3)
    Tm = Tsc / np.sqrt(msc[:, None, None] * msc[None, :, None] * msc[None, None, :])
    Nk = c.n_k
    L = np.array([[l0, l1, l2] for l0 in range(3) for l1 in range(2) for l2 in range(2)], float)
    U = np.zeros((Nk, sc.n_modes, c.n_modes), complex)
    for k in range(Nk):
        ph_l = np.exp(-2j * np.pi * (L @ ph.q[k])) / np.sqrt(Nk)      # (cells,)
        U[k] = np.kron(ph_l[:, None], ph.eigvec[k])                   # rows: (cell, atom, alpha)
    return c, ph, Tm, U


def _k_of(ph, m):
    return P.k_index(m, ph.grid)


def test_real_space_sum_equals_phi_plus_and_momentum_conservation(crystal_322):
    c, ph, Tm, U = crystal_322
    rng = np.random.default_rng(1)
    Nk = c.n_k
    for _ in range(6):
        k, kp = rng.integers(0, Nk, size=2)
        mk, mp = P.k_integer(k, ph.grid), P.k_integer(kp, ph.grid)
        kpp = _k_of(ph, [mk[i] + mp[i] for i in range(3)])
        Vsc = np.einsum('abc,as,bt,cu->stu', Tm, U[k], U[kp], U[kpp].conj(), optimize=True)
        phi, kpps = A.projection(c, ph, k, +1, kps=[kp])
        assert kpps[0] == kpp
        scale = np.abs(phi).max()
        assert np.allclose(Vsc * np.sqrt(Nk), phi[0], atol=1e-10 * scale)
        # any other k'' breaks momentum conservation: the real-space sum vanishes
        other = (kpp + 1 + rng.integers(0, Nk - 1)) % Nk
        Vbad = np.einsum('abc,as,bt,cu->stu', Tm, U[k], U[kp], U[other].conj(), optimize=True)
        assert np.abs(Vbad).max() < 1e-10 * scale


def test_real_space_sum_equals_phi_minus(crystal_322):
    c, ph, Tm, U = crystal_322
    rng = np.random.default_rng(2)
    Nk = c.n_k
    for _ in range(6):
        k, kp = rng.integers(0, Nk, size=2)
        mk, mp = P.k_integer(k, ph.grid), P.k_integer(kp, ph.grid)
        kpp = _k_of(ph, [mk[i] - mp[i] for i in range(3)])
        Vsc = np.einsum('abc,as,bt,cu->stu', Tm, U[k], U[kp].conj(), U[kpp].conj(), optimize=True)
        phi, kpps = A.projection(c, ph, k, -1, kps=[kp])
        assert kpps[0] == kpp
        assert np.allclose(Vsc * np.sqrt(Nk), phi[0], atol=1e-10 * np.abs(phi).max())


def test_permutation_identities_of_projection():
    c = diamond_si(grid=(3, 3, 3), rc3=4.0, masses=(M_SI, M_GE), seed=5)
    ph = P.phonons(c, velocities=False)
    rng = np.random.default_rng(4)
    for _ in range(8):
        k, kp = rng.integers(0, c.n_k, size=2)
        mk, mp = P.k_integer(k, ph.grid), P.k_integer(kp, ph.grid)
        kpp = _k_of(ph, [mk[i] + mp[i] for i in range(3)])
        a = A.projection(c, ph, k, +1, kps=[kp])[0][0]                 # phi+_{mu mu' mu''}
        b = A.projection(c, ph, kp, +1, kps=[k])[0][0]                 # phi+_{mu' mu mu''}
        d = A.projection(c, ph, kpp, -1, kps=[k])[0][0]                # phi-_{mu'' mu mu'}
        scale = np.abs(a).max()
        assert np.allclose(np.abs(a), np.abs(np.transpose(b, (1, 0, 2))), atol=1e-11 * scale)
        assert np.allclose(np.abs(a), np.abs(np.transpose(d, (1, 2, 0))), atol=1e-11 * scale)


def test_acoustic_modes_at_gamma_do_not_couple():
    c = diamond_si(grid=(3, 3, 3), rc3=4.7, masses=(M_SI, M_GE), seed=9)
    ph = P.phonons(c, velocities=False)
    for sign in (+1, -1):
        V, _ = A.projection(c, ph, 0, sign)
        assert np.abs(V[:, :3]).max() < 1e-12 * np.abs(V[:, 3:]).max()


# ----------------------------------------------------------------------------
# scalings, symmetry, normalisation
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def diamond_333():
    c = diamond_si(grid=(3, 3, 3), rc3=4.0, masses=(M_SI, M_GE), seed=21)
    ph = P.phonons(c, velocities=False)
    return c, ph


def test_zero_fc3_gives_zero_linewidth(diamond_333):
    c, ph = diamond_333
    g = A.linewidths(c.with_fc3_scaled(0.0), ph, [300.0], 0.1)
    assert np.all(g == 0.0)


def test_linewidth_scales_exactly_as_fc3_squared(diamond_333):
    c, ph = diamond_333
    g1 = A.linewidths(c, ph, [100.0, 300.0], 0.1, k_subset=[0, 4, 13])
    g2 = A.linewidths(c.with_fc3_scaled(2.0), ph, [100.0, 300.0], 0.1, k_subset=[0, 4, 13])
    assert np.array_equal(g2, 4.0 * g1)
    g3 = A.linewidths(c.with_fc3_scaled(0.3), ph, [300.0], 0.1, k_subset=[4])
    assert np.allclose(g3, 0.09 * g1[1:, 1:2], rtol=1e-12)


def test_time_reversal_of_linewidths(diamond_333):
    c, ph = diamond_333
    g = A.linewidths(c, ph, [300.0], 0.1)
    for k in range(c.n_k):
        mk = P.k_integer(k, ph.grid)
        km = _k_of(ph, [-x for x in mk])
        assert np.allclose(g[0, k], g[0, km], rtol=1e-9, atol=1e-14)
    assert np.all(g[0, 0, :3] == 0.0)
    assert np.all(g[0][ph.mask] > 0.0)


def test_folded_supercell_gamma_point_reproduces_crystal_linewidths():
    c = diamond_si(grid=(2, 2, 2), rc3=2.6, masses=(M_SI, M_GE), seed=31)
    ph = P.phonons(c, velocities=False)
    g = A.linewidths(c, ph, [300.0], 0.5)[0]
    sc = fold(c)
    phs = P.phonons(sc, velocities=False)
    gs = A.linewidths(sc, phs, [300.0], 0.5)[0, 0]
    nu_c = ph.nu[ph.mask]
    nu_s = phs.nu[0][phs.mask[0]]
    assert np.allclose(np.sort(nu_c), np.sort(nu_s), atol=1e-9)
    gc = g[ph.mask]
    gsv = gs[phs.mask[0]]
    order = np.argsort(nu_c)
    nu_sorted = nu_c[order]
    groups = np.split(order, np.nonzero(np.diff(nu_sorted) > 1e-6)[0] + 1)
    order_s = np.argsort(nu_s)
    groups_s = np.split(order_s, np.nonzero(np.diff(nu_s[order_s]) > 1e-6)[0] + 1)
    assert len(groups) == len(groups_s)
    for G, Gs in zip(groups, groups_s):
        assert len(G) == len(Gs)
        assert np.sum(gsv[Gs]) == pytest.approx(np.sum(gc[G]), rel=1e-9)


def test_sparse_gamma_path_matches_dense():
    sc = sige_supercell(reps=1, rc3=4.0)
    ph = P.phonons(sc, velocities=False)
    dense = A.linewidths(sc, ph, [100.0, 300.0], 0.1, average=False)[:, 0]
    sparse = A.linewidths_gamma_sparse(sc, ph, [100.0, 300.0], 0.1)
    assert np.allclose(sparse, dense, rtol=1e-10, atol=1e-14 * np.abs(dense).max())


def test_occupation_limits():
    w = np.array([0.5, 5.0, 50.0])
    T = 5000.0
    x = HBAR * w / (KB * T)
    n = A.occupation(w, T)
    # high-T series of 1/(e^x - 1)
    assert np.allclose(n, 1 / x - 0.5 + x / 12 - x ** 3 / 720, rtol=1e-7)
    T = 5.0
    x = HBAR * w / (KB * T)
    n = A.occupation(w[1:], T)
    assert np.allclose(n, np.exp(-x[1:]) * (1 + np.exp(-x[1:])), rtol=1e-6)
    assert np.allclose(A.occupation(w, 300.0, 'classical') * HBAR * w, KB * 300.0)
