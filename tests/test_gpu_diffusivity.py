"""Mode diffusivity at Gamma (kaldo_mode_diffusivity) through the C ABI against
the FP64 oracle.  Each side uses its own linewidths (the GPU's from
kaldo_linewidths, the oracle's from its own projection), so the comparison
covers the whole path.  The diffusivity's relative sensitivity to a relative
error in gamma is at most 1 (tau = g / (dw^2 + g^2)), so the bar is the
linewidth bar of the precision plus rounding: 1e-9 for FP64 linewidths and
1e-5 for FP32, relative to the largest D of each direction."""

import sys

import numpy as np
import pytest

from gen import diamond_si, random_crystal
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A, conductivity as C
from tests.supercell import fold

pytestmark = pytest.mark.gpu

T = [150.0, 600.0]
SIGMA = 0.3
TOL = {"fp64": 1e-9, "fp32": 1e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "folded-16at-gamma": lambda: fold(diamond_si(grid=(2, 2, 2), rc3=4.0, masses=(M_SI, M_GE), seed=17)),
    "random-7at-gamma": lambda: random_crystal(7, 3, np.random.default_rng(707)).with_grid((1, 1, 1)),
}
_ORACLE = {}


def _oracle(name):
    if name not in _ORACLE:
        c = CASES[name]()
        ph = P.phonons(c, velocities=False)
        _say(f"oracle: {name}")
        g = A.linewidths(c, ph, T, SIGMA)
        _ORACLE[name] = (c, ph, C.mode_diffusivity(c, ph, g))
    return _ORACLE[name]


@pytest.mark.parametrize("name,precision", [(n, p) for n in CASES for p in ("fp64", "fp32")])
def test_mode_diffusivity_against_oracle(name, precision):
    from paper_2009_01967_amd import kaldo
    c, ph, d_ref = _oracle(name)
    _say(f"case: {name}, {precision} linewidths")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.linewidths(c, T=T, sigma_thz=SIGMA, precision=precision)
        d = ctx.mode_diffusivity()
    assert d.shape == d_ref.shape
    scale = np.abs(d_ref).max(axis=(0, 1))
    assert (scale > 0).all()
    err = float((np.abs(d - d_ref).max(axis=(0, 1)) / scale).max())
    _say(f"  error {err:.3e} (tolerance {TOL[precision]:.0e})")
    assert err < TOL[precision], err
    assert np.all(d[:, ~ph.mask[0], :] == 0.0)


def test_mode_diffusivity_errors():
    """ESTATE before linewidths, EINVAL on a k grid and for a NULL output."""
    from paper_2009_01967_amd import kaldo
    c = CASES["random-7at-gamma"]()
    out = np.zeros((len(T), c.n_modes, 3))
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        assert kaldo.kaldo_mode_diffusivity(ctx.h, out) == kaldo.KALDO_ESTATE
        ctx.linewidths(c, T=T, sigma_thz=SIGMA, precision="fp64")
        assert kaldo.kaldo_mode_diffusivity(ctx.h, None) == kaldo.KALDO_EINVAL
    k = diamond_si(grid=(2, 2, 2), rc3=2.6, seed=3)
    with kaldo.Context(0) as ctx:
        ctx.phonons(k)
        ctx.linewidths(k, T=T, sigma_thz=SIGMA, precision="fp64")
        out = np.zeros((len(T), k.n_modes, 3))
        assert kaldo.kaldo_mode_diffusivity(ctx.h, out) == kaldo.KALDO_EINVAL
