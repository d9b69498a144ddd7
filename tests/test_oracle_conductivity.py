"""Pins of the oracle's heat capacities and conductivities: the defining
derivative of c, classical limits, limits of the generalised heat capacity,
antisymmetry of the generalised velocity, and QHGK on a folded crystal
supercell reducing to the RTA of the crystal as the linewidths go to zero."""

import numpy as np
import pytest

from gen import diamond_si
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A, conductivity as C, units
from tests.supercell import fold

HBAR = 6.582119569e-4
KB = 8.617333262e-5


def test_heat_capacity_is_temperature_derivative_of_energy():
    w = np.array([0.3, 3.0, 30.0, 90.0])
    for T in (20.0, 300.0, 1500.0):
        h = 1e-3 * T
        dn = (A.occupation(w, T + h) - A.occupation(w, T - h)) / (2 * h)
        assert np.allclose(C.heat_capacity(w, T), HBAR * w * dn, rtol=1e-7)


def test_heat_capacity_classical_limits():
    w = np.array([1.0, 10.0, 60.0])
    assert np.allclose(C.heat_capacity(w, 1e6), KB, rtol=1e-6)
    assert np.all(C.heat_capacity(w, 300.0, 'classical') == KB)
    assert np.all(C.generalized_heat_capacity(w, 300.0, 'classical') == KB)


def test_generalized_heat_capacity_limits_and_sign():
    w = np.array([5.0, 5.0 * (1 + 1e-7), 20.0, 70.0])
    T = 300.0
    c2 = C.generalized_heat_capacity(w, T)
    assert np.all(c2 > 0)
    assert np.allclose(np.diag(c2), C.heat_capacity(w, T), rtol=1e-12)
    assert c2[0, 1] == pytest.approx(C.heat_capacity(np.array([5.0]), T)[0], rel=1e-6)
    assert np.allclose(c2, c2.T, rtol=1e-12)
    # quantum -> classical at high T
    c_hot = C.generalized_heat_capacity(w, 1e6)
    assert np.allclose(c_hot, KB, rtol=1e-6)


def test_lorentzian_diagonal_is_rta_lifetime():
    w = np.array([1.0, 2.0, 3.0])
    g = np.array([0.1, 0.02, 0.3])
    tau = C.lorentzian_lifetime(w, g)
    assert np.allclose(np.diag(tau), 1.0 / (2.0 * g))


@pytest.fixture(scope="module")
def folded():
    c = diamond_si(grid=(3, 3, 3), rc3=2.6, masses=(M_SI, M_GE), seed=41)
    ph = P.phonons(c)
    sc = fold(c)
    phs = P.phonons(sc)
    return c, ph, sc, phs


def test_generalized_velocity_antisymmetric(folded):
    _, _, sc, phs = folded
    v = C.generalized_velocity(sc, phs)
    assert np.allclose(v, -np.transpose(v, (0, 2, 1)).conj(), atol=1e-10 * np.abs(v).max())
    assert np.abs(np.imag(v)).max() < 1e-12 * np.abs(v).max()


@pytest.mark.parametrize("scale", [1e-4, 1e-6])
def test_qhgk_on_folded_crystal_reduces_to_rta(folded, scale):
    c, ph, sc, phs = folded
    T = [300.0]

    def gfun(w):          # linewidths that depend on frequency only
        return scale * (0.2 + 0.01 * w + 1e-3 * w * w)

    g_c = np.where(ph.mask, gfun(ph.omega), 0.0)[None]
    g_s = np.where(phs.mask, gfun(phs.omega), 0.0)[None]
    k_rta = C.kappa_rta(c, ph, g_c, T)[0]
    k_qhgk = C.kappa_qhgk(sc, phs, g_s, T)[0]
    # off-diagonal Lorentzian terms are O(gamma^2 / dw^2) relative
    tol = 50 * scale + 1e-9
    assert np.allclose(k_qhgk, k_rta, rtol=tol, atol=tol * np.abs(k_rta).max())


def test_rta_kappa_scales_as_inverse_fc3_squared():
    c = diamond_si(grid=(3, 3, 3), rc3=2.6, seed=3)
    ph = P.phonons(c)
    g = A.linewidths(c, ph, [300.0], 0.2)
    g3 = A.linewidths(c.with_fc3_scaled(3.0), ph, [300.0], 0.2)
    k1 = C.kappa_rta(c, ph, g, [300.0])
    k3 = C.kappa_rta(c, ph, g3, [300.0])
    assert np.allclose(k3 * 9.0, k1, rtol=1e-12)
    assert np.all(np.linalg.eigvalsh(k1[0]) > 0)


def test_rta_kappa_classical_capacity_is_kb():
    c = diamond_si(grid=(3, 3, 3), rc3=2.6, seed=3)
    ph = P.phonons(c)
    g = np.where(ph.mask, 0.01, 0.0)[None]
    kc = C.kappa_rta(c, ph, g, [300.0], stats='classical')[0]
    # classical: kappa = k_B / (2 gamma) * sum vv / (N_k V)
    V = abs(np.linalg.det(c.cell))
    expect = KB / 0.02 * np.einsum('ksab->ab', ph.vv) / (ph.n_k * V) * 1.602176634e3
    assert np.allclose(kc, expect, rtol=1e-12)


def test_diffusivity_sums_to_classical_qhgk_kappa(folded):
    """With c = k_B for every pair (classical limit), the QHGK conductivity is
    k_B / V times the summed mode diffusivities: k_B sum_mu D_mu,a = V kappa_aa."""
    _, _, sc, phs = folded
    rng = np.random.default_rng(7)
    g = np.where(phs.mask, 0.05 + 0.2 * rng.random(phs.omega.shape), 0.0)[None]
    D = C.mode_diffusivity(sc, phs, g)[0]                       # (n, 3) mm^2/s
    k = C.kappa_qhgk(sc, phs, g, [300.0], stats="classical")[0]
    lhs = units.KB * D.sum(axis=0) * 1e2 * units.KAPPA_TO_SI   # back to A^2/ps
    rhs = C.volume(sc) * np.diag(k)
    assert np.allclose(lhs, rhs, rtol=1e-12), (lhs, rhs)
    assert (D >= 0).all()
    assert np.all(D[~phs.mask[0]] == 0.0)


@pytest.mark.parametrize("scale", [1e-4, 1e-6])
def test_diffusivity_on_folded_crystal_matches_group_velocities(folded, scale):
    """In a folded supercell with small linewidths that depend on frequency
    only, the off-diagonal Lorentzian terms vanish as (gamma / dw)^2 and the
    summed diffusivity tends to sum_{k,s} v_ks,a^2 / (2 gamma_ks) of the
    primitive crystal, which its classical RTA conductivity carries:
    sum_mu D_mu,a = N_k V kappa_RTA,aa / k_B."""
    c, ph, sc, phs = folded

    def gfun(w):
        return scale * (0.2 + 0.01 * w + 1e-3 * w * w)

    g_c = np.where(ph.mask, gfun(ph.omega), 0.0)[None]
    g_s = np.where(phs.mask, gfun(phs.omega), 0.0)[None]
    D = C.mode_diffusivity(sc, phs, g_s)[0]
    k_rta = C.kappa_rta(c, ph, g_c, [300.0], stats="classical")[0]
    lhs = D.sum(axis=0) * 1e2
    rhs = c.n_k * C.volume(c) * np.diag(k_rta) / (units.KB * units.KAPPA_TO_SI)
    tol = 50 * scale + 1e-9
    assert np.allclose(lhs, rhs, rtol=tol), (lhs, rhs)


# ---- the Lorentzian generalised lifetime off the diagonal (Sec. II.C, eq. lorentzian_amorphous)

def test_lorentzian_half_maximum_at_summed_linewidths():
    """As a function of the frequency gap, tau_{mu mu'} peaks at 1/(gamma + gamma')
    and falls to half of that where |w - w'| = gamma + gamma': this fixes the
    scale of the gap against the linewidths."""
    for a, b in ((0.3, 0.1), (0.05, 2.0), (1.0, 1.0)):
        g = a + b
        w = np.array([7.0, 7.0, 7.0 + g, 7.0 - g])
        gam = np.array([a, b, b, b])
        tau = C.lorentzian_lifetime(w, gam)
        assert tau[0, 1] == pytest.approx(1.0 / g, rel=1e-14)       # zero gap: the peak
        assert tau[0, 2] == pytest.approx(0.5 / g, rel=1e-14)       # gap +g: half maximum
        assert tau[0, 3] == pytest.approx(0.5 / g, rel=1e-14)       # gap -g
        assert np.allclose(tau, tau.T, rtol=1e-15)


def test_lorentzian_area_over_the_gap_is_pi():
    """Integrated over the gap w - w' on a dense grid, tau_{mu mu'} has area
    2 arctan(L / g) over [-L, L] (-> pi): its normalisation as a line shape."""
    a, b = 0.2, 0.35
    g = a + b
    L = 50.0 * g
    x = np.linspace(-L, L, 4001)
    w = np.concatenate(([0.0], x))
    gam = np.concatenate(([a], np.full(x.size, b)))
    tau = C.lorentzian_lifetime(w, gam)[0, 1:]
    h = x[1] - x[0]
    area = h * (tau.sum() - 0.5 * (tau[0] + tau[-1]))              # trapezoid rule
    assert area == pytest.approx(2.0 * np.arctan(L / g), rel=1e-9)
    assert area == pytest.approx(np.pi, rel=2.0 / 50.0)


def _two_mode_cell():
    """One atom (mass 4 amu) in a cubic 5 A cell with fc2 blocks on the +x and
    -x images: B = 0.3 eV/A^2 in entry (x, y) for R = +x, its transpose for
    R = -x.  The displacement Hessian of the generalised velocity is then
    M_x[0][1] = -5 * 0.3 / 4 and M_x[1][0] = +5 * 0.3 / 4 (in eV/(A amu)),
    and zero elsewhere."""
    from gen.crystals import Crystal
    B = np.zeros((3, 3))
    B[0, 1] = 0.3
    return Crystal(
        name="two-mode", cell=5.0 * np.eye(3), positions=np.zeros((1, 3)), masses=np.array([4.0]),
        fc2_i=np.array([0, 0], np.int32), fc2_j=np.array([0, 0], np.int32),
        fc2_R=np.array([[1, 0, 0], [-1, 0, 0]], np.int32), fc2_val=np.stack([B, B.T]),
        fc3_i=np.zeros(0, np.int32), fc3_j=np.zeros(0, np.int32), fc3_l=np.zeros(0, np.int32),
        fc3_R1=np.zeros((0, 3), np.int32), fc3_R2=np.zeros((0, 3), np.int32),
        fc3_val=np.zeros((0, 3, 3, 3)), grid=(1, 1, 1))


def _two_mode_phonons():
    """Modes 10, 12 and 30 rad/ps with the unit vectors as eigenvectors."""
    w = np.array([[10.0, 12.0, 30.0]])
    return P.Phonons(grid=(1, 1, 1), q=np.zeros((1, 3)), omega=w, eigvec=np.eye(3, dtype=complex)[None],
                     mask=np.ones((1, 3), bool), sets=[[np.array([0]), np.array([1]), np.array([2])]],
                     velocity=np.zeros((1, 3, 3)), vv=np.zeros((1, 3, 3, 3)))


def test_hand_worked_two_mode_qhgk_and_diffusivity():
    """Worked by hand: v_{01x} = M_x[0][1] / (2 sqrt(10 * 12)) = -1.5 eV / (8 sqrt(120)),
    with gamma = (0.5, 1.5, 0.2) rad/ps the pair lifetime is
    tau_01 = 2 / ((10 - 12)^2 + 2^2) = 0.25 ps (the gap equals the summed
    linewidths, so the off-diagonal Lorentzian is at half maximum).  The only
    nonzero velocities are v_01 = -v_10, so in the classical limit
    kappa_xx = 2 k_B tau_01 v_01^2 / V and D_0x = D_1x = v_01^2 tau_01."""
    c, ph = _two_mode_cell(), _two_mode_phonons()
    g = np.array([[[0.5, 1.5, 0.2]]])
    v01 = 1.5 * units.EV_IN_AMU_A2_PS2 / (8.0 * np.sqrt(120.0))      # A/ps
    k = C.kappa_qhgk(c, ph, g, [300.0], stats="classical")[0]
    expect = 2.0 * units.KB * 0.25 * v01 ** 2 / 125.0 * units.KAPPA_TO_SI
    assert k[0, 0] == pytest.approx(expect, rel=1e-13)
    assert np.abs(k.ravel()[1:]).max() < 1e-13 * expect
    D = C.mode_diffusivity(c, ph, g)[0]
    assert D[0, 0] == pytest.approx(v01 ** 2 * 0.25 * 1e-2, rel=1e-13)
    assert D[1, 0] == pytest.approx(v01 ** 2 * 0.25 * 1e-2, rel=1e-13)
    assert np.abs(D[2]).max() == 0.0 and np.abs(D[:, 1:]).max() == 0.0


# ---- the QHGK options of Appendix A: a bandwidth (Allen-Feldman) and an energy threshold

def test_hand_worked_bandwidth_replaces_every_linewidth():
    """With a bandwidth eta = 0.5 rad/ps every linewidth is eta, so the pair
    width is 2 eta = 1 and tau_01 = 1 / ((10 - 12)^2 + 1) = 0.2 ps, whatever
    linewidths are passed; the diagonal lifetime is 1 / (2 eta) = 1 ps."""
    c, ph = _two_mode_cell(), _two_mode_phonons()
    v01 = 1.5 * units.EV_IN_AMU_A2_PS2 / (8.0 * np.sqrt(120.0))
    for g in (np.array([[[0.5, 1.5, 0.2]]]), np.array([[[3.0, 0.01, 7.0]]])):
        k = C.kappa_qhgk(c, ph, g, [300.0], stats="classical", bandwidth=0.5)[0]
        assert k[0, 0] == pytest.approx(2.0 * units.KB * 0.2 * v01 ** 2 / 125.0 * units.KAPPA_TO_SI, rel=1e-13)
        D = C.mode_diffusivity(c, ph, g, bandwidth=0.5)[0]
        assert D[0, 0] == pytest.approx(v01 ** 2 * 0.2 * 1e-2, rel=1e-13)
    tau = C.lorentzian_lifetime(np.array([1.0, 4.0]), np.array([9.0, 9.0]), bandwidth=0.25)
    assert np.allclose(np.diag(tau), 2.0)
    assert tau[0, 1] == pytest.approx(0.5 / (9.0 + 0.25), rel=1e-14)


def test_hand_worked_threshold_drops_pairs_beyond_the_gap():
    """The one coupled pair has the gap |10 - 12| = 2 rad/ps: a threshold of
    1.5 drops it (kappa = D = 0), a threshold of exactly 2 keeps it."""
    c, ph = _two_mode_cell(), _two_mode_phonons()
    g = np.array([[[0.5, 1.5, 0.2]]])
    assert np.abs(C.kappa_qhgk(c, ph, g, [300.0], stats="classical", threshold=1.5)).max() == 0.0
    assert np.abs(C.mode_diffusivity(c, ph, g, threshold=1.5)).max() == 0.0
    k_all = C.kappa_qhgk(c, ph, g, [300.0], stats="classical")
    assert np.array_equal(C.kappa_qhgk(c, ph, g, [300.0], stats="classical", threshold=2.0), k_all)
    w = np.array([1.0, 2.0, 4.5, 4.6])
    tau = C.lorentzian_lifetime(w, np.full(4, 0.1), threshold=1.0)
    kept = np.abs(w[:, None] - w[None, :]) <= 1.0
    assert np.array_equal(tau > 0, kept)                 # brute force over the 16 pairs


def test_threshold_above_the_spectrum_changes_nothing(folded):
    """A threshold wider than the whole spectrum keeps every pair: bitwise the
    conductivity and diffusivity without one."""
    c, ph, sc, phs = folded
    rng = np.random.default_rng(5)
    g = rng.uniform(0.05, 0.5, size=(1, 1, sc.n_modes))
    wmax = phs.omega.max() * 1.01
    assert np.array_equal(C.kappa_qhgk(sc, phs, g, [300.0], threshold=wmax), C.kappa_qhgk(sc, phs, g, [300.0]))
    assert np.array_equal(C.mode_diffusivity(sc, phs, g, threshold=wmax), C.mode_diffusivity(sc, phs, g))


def test_threshold_splits_the_classical_sum_rule(folded):
    """k_B sum_mu D_mu,a = V kappa_aa holds pair by pair, so it holds with any
    threshold, and kappa falls monotonically as the threshold narrows (every
    classical term c tau v^2 is >= 0)."""
    c, ph, sc, phs = folded
    rng = np.random.default_rng(6)
    g = rng.uniform(0.05, 0.5, size=(1, 1, sc.n_modes))
    prev = np.inf
    for thr in (80.0, 10.0, 3.0, 0.5):
        k = C.kappa_qhgk(sc, phs, g, [300.0], stats="classical", threshold=thr)[0]
        D = C.mode_diffusivity(sc, phs, g, threshold=thr)[0]
        lhs = units.KB * D.sum(axis=0) * 1e2
        rhs = C.volume(sc) * np.diag(k) / units.KAPPA_TO_SI
        assert np.allclose(lhs, rhs, rtol=1e-10)
        assert np.trace(k) <= prev * (1 + 1e-12)
        prev = np.trace(k)
