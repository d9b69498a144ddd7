"""Adaptive delta widths (kaldo_adaptive_width, Appendix A) through the C ABI
against the FP64 oracle: the few-branch kernel (diamond, 6 branches) and the
crystal GEMM path (a 4-atom cell, 12 branches), every mode, in FP64, FP32 and
BF16X3, with the RTA conductivity; a vanishing scale gives the fixed width;
the calls that refuse adaptive widths."""

import sys

import numpy as np
import pytest

from gen import diamond_si, random_crystal, sige_supercell
from oracle import phonons as P, anharmonic as A, conductivity as C
from tests.parity import TOL, gamma_error, kappa_error

pytestmark = pytest.mark.gpu

T = [300.0, 800.0]
SIGMA = 0.05
SCALE = 1.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "diamond-2at-4^3": lambda: diamond_si(grid=(4, 4, 4), rc3=2.6),
    "random-4at-3x3x2": lambda: random_crystal(4, 3, np.random.default_rng(404)).with_grid((3, 3, 2)),
}
_REF = {}


def _oracle(name):
    if name not in _REF:
        c = CASES[name]()
        ph = P.phonons(c)
        _say(f"oracle: {name}, adaptive scale {SCALE}")
        g = A.linewidths(c, ph, T, SIGMA, adaptive=SCALE)
        _REF[name] = (c, ph, g, C.kappa_rta(c, ph, g, T))
    return _REF[name]


@pytest.mark.parametrize("name,precision", [(n, p) for n in CASES for p in ("fp64", "fp32", "bf16x3")
                                            if not (n.startswith("diamond") and p == "bf16x3")])
def test_adaptive_linewidths_against_oracle(name, precision):
    from paper_2009_01967_amd import kaldo
    c, ph, g_ref, k_ref = _oracle(name)
    _say(f"case: {name}, adaptive widths, {precision}")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.adaptive_width(SCALE)
        g = ctx.linewidths(c, T=T, sigma_thz=SIGMA, precision=precision)
        k = ctx.kappa_rta()
        ctx.adaptive_width(0.0)
        g_fixed = ctx.linewidths(None, T=T, sigma_thz=SIGMA, precision=precision)
    eg, ek = gamma_error(g, g_ref, ph.mask), kappa_error(k, k_ref)
    _say(f"  gamma error {eg:.3e}, kappa error {ek:.3e} (tolerance {TOL[precision]:.0e})")
    assert eg < TOL[precision], eg
    assert ek < TOL[precision], ek
    # the widths matter: adaptive and fixed linewidths differ well beyond the tolerance
    assert gamma_error(g_fixed, g_ref, ph.mask) > 100 * TOL[precision]


def test_vanishing_scale_gives_the_fixed_width():
    from paper_2009_01967_amd import kaldo
    c = CASES["random-4at-3x3x2"]()
    _say("case: adaptive scale 1e-12 against fixed widths, fp64")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        g0 = ctx.linewidths(c, T=T, sigma_thz=SIGMA, precision="fp64")
        ctx.adaptive_width(1e-12)
        g1 = ctx.linewidths(None, T=T, sigma_thz=SIGMA, precision="fp64")
    ph = P.phonons(c, velocities=False)
    assert gamma_error(g1, g0, ph.mask) < 1e-12


def test_adaptive_width_errors():
    from paper_2009_01967_amd import kaldo
    c = diamond_si(grid=(3, 3, 3), rc3=2.6)
    with kaldo.Context(0) as ctx:
        assert kaldo.kaldo_adaptive_width(ctx.h, -1.0) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_adaptive_width(ctx.h, float("nan")) == kaldo.KALDO_EINVAL
        ctx.phonons(c)
        ctx.adaptive_width(1.0)
        with pytest.raises(kaldo.KaldoError):
            ctx.linewidths(c, T=[300.0], sigma_thz=0.1, delta="lorentz")
        ctx.linewidths(c, T=[300.0], sigma_thz=0.1)
        out = np.zeros((1, 3, 3))
        assert kaldo.kaldo_kappa_bte(ctx.h, 0, 10, 1e-10, out) == kaldo.KALDO_EINVAL
        ctx.adaptive_width(0.0)
        ctx.linewidths(None, T=[300.0], sigma_thz=0.1)
        kaldo._check(ctx.h, kaldo.kaldo_kappa_bte(ctx.h, 0, 10, 1e-10, out))
    g = sige_supercell(reps=1)
    with kaldo.Context(0) as ctx:
        ctx.phonons(g)
        ctx.adaptive_width(1.0)
        with pytest.raises(kaldo.KaldoError):
            ctx.linewidths(g, T=[300.0], sigma_thz=0.1)
