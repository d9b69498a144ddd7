"""Phase space per mode (kaldo_phase_space) through the C ABI against the FP64
oracle, for the three delta kinds and both statistics, on a crystal grid, a
4-atom cell and at Gamma; argument errors; and that the call leaves the state
of kaldo_kappa_* alone."""

import sys

import numpy as np
import pytest

from gen import diamond_si, random_crystal, workload
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A
from tests.supercell import fold

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _err(g, ref):
    ref = np.asarray(ref)
    floor = 1e-6 * np.abs(ref).max()
    return float(np.max(np.abs(g - ref) / np.maximum(np.abs(ref), floor)))


CRYSTALS = {
    "diamond-4x4x4": lambda: workload("diamond-2at-4x4x4-shell1"),
    "four-atom-3x3x2": lambda: random_crystal(4, 3, np.random.default_rng(404)).with_grid((3, 3, 2)),
    "folded-16at-gamma": lambda: fold(diamond_si(grid=(2, 2, 2), rc3=4.0, masses=(M_SI, M_GE), seed=17)),
}
CASES = [("diamond-4x4x4", "gauss", "quantum", [0.0, 300.0], 0.1),
         ("diamond-4x4x4", "lorentz", "classical", [300.0, 900.0], 0.2),
         ("diamond-4x4x4", "triangle", "quantum", [600.0], 0.3),
         ("four-atom-3x3x2", "gauss", "quantum", [150.0, 600.0], 0.3),
         ("four-atom-3x3x2", "lorentz", "quantum", [300.0], 0.3),
         ("folded-16at-gamma", "gauss", "quantum", [100.0, 300.0], 0.3),
         ("folded-16at-gamma", "triangle", "classical", [300.0], 0.5)]


@pytest.mark.parametrize("name,delta,stats,T,sigma", CASES)
def test_phase_space_against_oracle(name, delta, stats, T, sigma):
    from paper_2009_01967_amd import kaldo
    c = CRYSTALS[name]()
    _say(f"case: {name}, {delta}, {stats}, T={T}, sigma={sigma}")
    ph = P.phonons(c, velocities=False)
    ref = A.phase_space(ph, T, sigma, stats=stats, delta=delta)
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        g = ctx.phase_space(T=T, sigma_thz=sigma, classical=stats == "classical", delta=delta)
    assert np.all(g[:, ~ph.mask] == 0.0)
    err = _err(g, ref)
    _say(f"  error {err:.3e} (tolerance {TOL:.0e})")
    assert err < TOL, err


def test_phase_space_errors_and_state():
    from paper_2009_01967_amd import kaldo
    c = workload("diamond-2at-4x4x4-shell1")
    _say("case: phase space errors, kappa state kept")
    with kaldo.Context(0) as ctx:
        g = np.zeros((1, c.n_k, c.n_modes))
        assert kaldo.kaldo_phase_space(ctx.h, [300.0], 0.1, g_out=g) == kaldo.KALDO_ESTATE
        ctx.phonons(c)
        assert kaldo.kaldo_phase_space(ctx.h, [300.0], 0.1, g_out=None) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_phase_space(ctx.h, [300.0], -0.1, g_out=g) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_phase_space(ctx.h, [300.0], 0.1, delta=9, g_out=g) == kaldo.KALDO_EINVAL
        ctx.linewidths(c, T=[300.0], sigma_thz=0.1)
        k0 = ctx.kappa_rta()
        ctx.phase_space(T=[100.0, 200.0, 400.0], sigma_thz=0.3, delta="lorentz")
        k1 = ctx.kappa_rta()
    assert np.array_equal(k0, k1)
