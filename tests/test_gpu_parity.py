"""GPU path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 1e-10, FP32 1e-5 relative (gamma: max over unmasked modes
of |g - g_ref| / max(g_ref, 1e-6 max g_ref) after degenerate-set averaging;
kappa: Frobenius relative error)."""

import sys

import numpy as np
import pytest

from gen import diamond_si, WORKLOADS, workload
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A
from tests.parity import TOL, gamma_error, kappa_error, oracle_all

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2009_01967_amd import kaldo
    return kaldo.Context(0)


def _ok(err, tol):
    print(f"  error {err:.3e} (tolerance {tol:.0e})", flush=True)
    assert err < tol, err


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small_diamond():
    w = WORKLOADS["diamond-2at-4x4x4-shell1"]
    c = workload("diamond-2at-4x4x4-shell1")
    ph, g, k = oracle_all(c, w["T"], w["sigma_thz"])
    return c, w, ph, g, k


def test_phonon_frequencies_and_velocities(small_diamond):
    c, w, ph, g, k = small_diamond
    _say("case: diamond 4x4x4 phonons")
    with _ctx() as ctx:
        nu = ctx.phonons(c)
        vel = np.zeros((c.n_k, c.n_modes, 3))
        ctx.phonons(None, c.grid, vel_out=vel)
    # eigenvalues nu^2 (signed) to FP64 eigensolver accuracy; zero modes are noise in nu itself
    lam = np.sign(nu) * nu ** 2
    lam_ref = np.sign(ph.nu) * ph.nu ** 2
    err = float(np.max(np.abs(lam - lam_ref)) / np.abs(lam_ref).max())
    assert err < 1e-12, err
    # velocities of non-degenerate modes are basis independent
    for kk in range(c.n_k):
        for S in ph.sets[kk]:
            if len(S) == 1 and ph.mask[kk, S[0]]:
                d = float(np.max(np.abs(vel[kk, S[0]] - ph.velocity[kk, S[0]])))
                assert d < 1e-9 * max(1.0, np.abs(ph.velocity).max()), (kk, S[0], d)


def test_two_species_eigenvalues_all_k():
    """Exact degeneracies at zone-boundary points with two masses (the batched
    Jacobi eigensolver must keep its matrix Hermitian to resolve them)."""
    c = diamond_si(grid=(4, 4, 4), rc3=2.6, masses=(M_SI, M_GE), seed=7)
    _say("case: two-species diamond 4x4x4 eigenvalues")
    ph = P.phonons(c, velocities=False)
    with _ctx() as ctx:
        nu = ctx.phonons(c)
    lam = np.sign(nu) * nu ** 2
    lam_ref = np.sign(ph.nu) * ph.nu ** 2
    err = float(np.max(np.abs(lam - lam_ref)) / np.abs(lam_ref).max())
    print(f"  eigenvalue error {err:.3e}", flush=True)
    assert err < 1e-12, err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_linewidths_and_kappa_small_diamond(small_diamond, precision):
    c, w, ph, g, k = small_diamond
    _say(f"case: diamond 4x4x4 linewidths {precision}")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision=precision)
        kk = ctx.kappa_rta()
    _ok(gamma_error(gg, g, ph.mask), TOL[precision])
    _ok(kappa_error(kk, k), TOL[precision])
    assert np.all(gg[:, ~ph.mask] == 0.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_grid_two_species_several_temperatures(precision):
    # 3x4x5 = 60 points: one partial p-tile; second-shell fc3 with triangles
    c = diamond_si(grid=(3, 4, 5), rc3=4.0, masses=(M_SI, M_GE), seed=123)
    T = [50.0, 300.0, 1200.0, 0.0]
    _say(f"case: diamond 3x4x5 two species {precision}")
    ph, g, k = oracle_all(c, T[:3], 0.15)
    g0 = A.linewidths(c, ph, [0.0], 0.15)
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=T, sigma_thz=0.15, precision=precision)
        kk = ctx.kappa_rta()
    _ok(gamma_error(gg[:3], g, ph.mask), TOL[precision])
    _ok(gamma_error(gg[3:], g0, ph.mask), TOL[precision])
    _ok(kappa_error(kk[:3], k), TOL[precision])


def test_classical_statistics():
    c = diamond_si(grid=(4, 4, 4), rc3=2.6, masses=(M_SI, M_GE), seed=7)
    T = [300.0, 900.0]
    _say("case: diamond 4x4x4 classical fp64")
    ph, g, k = oracle_all(c, T, 0.1, stats="classical")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=T, sigma_thz=0.1, classical=True)
        kk = ctx.kappa_rta()
    _ok(gamma_error(gg, g, ph.mask), TOL["fp64"])
    _ok(kappa_error(kk, k), TOL["fp64"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_diamond_16_cubed_sampled_k(precision):
    """The benchmark workload at full size (16^3, 3rd-shell fc3, 3 T), in the
    benchmark's launch configuration; the oracle evaluates sampled k points."""
    name = "diamond-2at-16x16x16-shell3"
    w = WORKLOADS[name]
    c = workload(name)
    _say(f"case: {name} {precision}")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision=precision)
    ph = P.phonons(c, velocities=False)
    ks = [0, 1, 17, 273, 2080, 4095]   # Gamma, nearest neighbour of Gamma, generic, zone boundary
    g = A.linewidths(c, ph, w["T"], w["sigma_thz"], k_subset=ks)
    _ok(gamma_error(gg[:, ks], g, ph.mask[ks]), TOL[precision])
    assert np.all(gg[:, 0, :3] == 0.0)


def test_invariants_through_abi():
    """fc3 -> 0 gives 0; fc3 -> 2 fc3 gives exactly 4x; repeated runs are bitwise equal."""
    c = diamond_si(grid=(4, 4, 4), rc3=4.0, seed=11)
    _say("case: invariants fp64")
    with _ctx() as ctx:
        ctx.phonons(c)
        g1 = ctx.linewidths(c, T=[300.0], sigma_thz=0.1)
        g1b = ctx.linewidths(None, T=[300.0], sigma_thz=0.1)
        g2 = ctx.linewidths(c.with_fc3_scaled(2.0), T=[300.0], sigma_thz=0.1)
        g0 = ctx.linewidths(c.with_fc3_scaled(0.0), T=[300.0], sigma_thz=0.1)
    assert np.array_equal(g1, g1b)
    assert np.array_equal(g2, 4.0 * g1)
    assert np.all(g0 == 0.0)


def test_abi_errors():
    from paper_2009_01967_amd import kaldo
    c = diamond_si(grid=(2, 2, 2))
    _say("case: ABI errors")
    ctx = kaldo.Context(0)
    try:
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.linewidths(c)
        assert e.value.status == kaldo.KALDO_ESTATE
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.kappa_rta()
        assert e.value.status == kaldo.KALDO_ESTATE
        bad = c.with_grid((2, 2, 2))
        bad.fc2_j = bad.fc2_j.copy()
        bad.fc2_j[0] = 7
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.phonons(bad)
        assert e.value.status == kaldo.KALDO_EINVAL
        ctx.phonons(c)
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.linewidths(c, T=[300.0] * 9)
        assert e.value.status == kaldo.KALDO_EINVAL
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.linewidths(c, sigma_thz=0.0)
        assert e.value.status == kaldo.KALDO_EINVAL
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.kappa_qhgk()
        assert e.value.status in (kaldo.KALDO_ESTATE, kaldo.KALDO_EINVAL)
        assert kaldo.kaldo_set_tuning(ctx.h, 99) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_set_tuning(ctx.h, -1) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_FIXED) == kaldo.KALDO_OK
        assert kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_AUTO) == kaldo.KALDO_OK
        # a negative spring makes an imaginary mode
        uns = c.with_grid((2, 2, 2))
        uns.fc2_val = -uns.fc2_val
        with pytest.raises(kaldo.KaldoError) as e:
            ctx.phonons(uns)
        assert e.value.status == kaldo.KALDO_EUNSTABLE
        # the caller's input buffers are not retained: overwrite them and rerun
        c2 = c.with_grid((2, 2, 2))
        ctx.phonons(c2)
        g_a = ctx.linewidths(c2, T=[300.0], sigma_thz=0.2)
        c2.fc3_val[:] = np.nan
        c2.fc2_val[:] = np.nan
        g_b = ctx.linewidths(None, T=[300.0], sigma_thz=0.2)
        assert np.array_equal(g_a, g_b)
    finally:
        ctx.close()
