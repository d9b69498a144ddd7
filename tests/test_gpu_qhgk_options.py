"""QHGK stage at 648 modes and the QHGK options of Appendix A through the C
ABI against the FP64 oracle:

* the linewidths of every mode of the 216-atom SiGe cell (FP64, FP32,
  BF16X3) against the oracle's, stored in tests/golden/sige648.json by
  tests/golden/make_sige648.py;
* kappa_QHGK and the mode diffusivity from the GPU's FP64 linewidths against
  the oracle's from its own, at 1e-10 (kappa: relative Frobenius; D: element
  by element relative to each |D|), many u slices and the set averaging
  included;
* the bandwidth (Allen-Feldman: no linewidths at all) and the energy
  threshold, on the same installed linewidths on both sides;
* the linewidths interpolated in frequency (kaldo_gamma_interpolate) from the
  648-mode cell onto the 1536-mode one, and kappa_QHGK from them, against the
  oracle's interpolation; host and device source arrays give the same bits;
* errors of the new calls."""

import json
import os
import sys

import numpy as np
import pytest

from gen import sige_supercell, diamond_si
from oracle import phonons as P, conductivity as C, interpolation as I
from tests.devmem import DeviceArray
from tests.parity import gamma_error, kappa_error, set_average, TOL

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sige648.json")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_CACHE = {}


def _sige648():
    """The 648-mode cell, the oracle's phonons and its stored linewidths
    (set averaged with the oracle's sets)."""
    if "648" not in _CACHE:
        with open(GOLDEN) as f:
            gold = json.load(f)
        c = sige_supercell(reps=3)
        ph = P.phonons(c, velocities=False)
        m = ph.mask[0]   # the three acoustic modes at Gamma sit at rounding noise around 0
        assert np.allclose(ph.omega[0][m], np.asarray(gold["omega"])[m], rtol=1e-10, atol=0.0)
        g = set_average(ph, np.asarray(gold["gamma"])[:, None, :], [0])
        _CACHE["648"] = (c, ph, g, gold["T"], gold["sigma_thz"])
    return _CACHE["648"]


def _d_error(d, d_ref):
    """max |d - d_ref| / |d_ref| over the entries of unmasked modes (floor 1e-12 max|d_ref|)."""
    ref = np.abs(d_ref)
    floor = 1e-12 * ref.max()
    return float(np.max(np.abs(d - d_ref) / np.maximum(ref, floor)))


def _off_gaps(omega, thr):
    """A threshold nudged so that no frequency gap lies within 1e-7 of it."""
    gaps = np.abs(omega[:, None] - omega[None, :]).ravel()
    while np.min(np.abs(gaps - thr)) < 1e-7 * thr:
        thr *= 1.0 + 1e-5
    return thr


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_sige648_linewidths_against_oracle(precision):
    from paper_2009_01967_amd import kaldo
    c, ph, g_ref, T, sigma = _sige648()
    _say(f"case: sige-216at linewidths, {precision}")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        g = ctx.linewidths(c, T=T, sigma_thz=sigma, precision=precision)
    err = gamma_error(g, g_ref, ph.mask[0])
    _say(f"  gamma error {err:.3e} (tolerance {TOL[precision]:.0e})")
    assert err < TOL[precision], err
    assert np.all(g[:, 0, ~ph.mask[0]] == 0.0)


def test_sige648_kappa_and_diffusivity_against_oracle():
    """GPU gamma -> GPU kappa and D; oracle gamma -> oracle kappa and D."""
    from paper_2009_01967_amd import kaldo
    c, ph, g_ref, T, sigma = _sige648()
    _say("case: sige-216at kappa_QHGK and mode diffusivity, fp64")
    k_ref = C.kappa_qhgk(c, ph, g_ref, T)
    d_ref = C.mode_diffusivity(c, ph, g_ref)
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.linewidths(c, T=T, sigma_thz=sigma, precision="fp64")
        k = ctx.kappa_qhgk()
        d = ctx.mode_diffusivity()
    ek, ed = kappa_error(k, k_ref), _d_error(d, d_ref)
    _say(f"  kappa error {ek:.3e}, diffusivity error {ed:.3e}")
    assert ek < 1e-10, ek
    assert ed < 1e-10, ed
    assert np.all(d[:, ~ph.mask[0], :] == 0.0)


@pytest.mark.parametrize("bandwidth,threshold", [(0.0, 3.0), (0.0, 12.0), (0.4, 0.0), (0.4, 3.0)])
def test_qhgk_options_against_oracle(bandwidth, threshold):
    """The same installed linewidths on both sides; a bandwidth needs none (zeros installed)."""
    from paper_2009_01967_amd import kaldo
    c, ph, g_ref, T, sigma = _sige648()
    thr = _off_gaps(ph.omega[0], threshold) if threshold > 0 else 0.0
    bw = bandwidth if bandwidth > 0 else None
    _say(f"case: sige-216at QHGK options, bandwidth {bandwidth}, threshold {thr}")
    g_in = np.zeros_like(g_ref) if bw else g_ref
    k_ref = C.kappa_qhgk(c, ph, g_in, T, bandwidth=bw, threshold=thr if thr > 0 else None)
    d_ref = C.mode_diffusivity(c, ph, g_in, bandwidth=bw, threshold=thr if thr > 0 else None)
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.set_gamma(T=T, gamma=None if bw else g_ref)
        ctx.qhgk_options(bandwidth=bandwidth, threshold=thr)
        k = ctx.kappa_qhgk()
        d = ctx.mode_diffusivity()
    ek, ed = kappa_error(k, k_ref), _d_error(d, d_ref)
    _say(f"  kappa error {ek:.3e}, diffusivity error {ed:.3e}")
    assert ek < 1e-10, ek
    assert ed < 1e-10, ed


def test_threshold_wider_than_the_spectrum_is_bitwise_no_threshold():
    from paper_2009_01967_amd import kaldo
    c, ph, g_ref, T, sigma = _sige648()
    _say("case: sige-216at threshold above the spectrum")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.set_gamma(T=T, gamma=g_ref)
        k0, d0 = ctx.kappa_qhgk(), ctx.mode_diffusivity()
        ctx.qhgk_options(threshold=2.0 * ph.omega[0].max())
        k1, d1 = ctx.kappa_qhgk(), ctx.mode_diffusivity()
        ctx.qhgk_options(threshold=float("inf"))
        k2 = ctx.kappa_qhgk()
    assert np.array_equal(k0, k1) and np.array_equal(d0, d1) and np.array_equal(k0, k2)


def test_gamma_interpolate_onto_a_larger_cell_against_oracle():
    """Source: the 648-mode cell's oracle frequencies and linewidths; target:
    the 512-atom cell (1536 modes).  The interpolated linewidths and kappa_QHGK
    from them, GPU against oracle."""
    from paper_2009_01967_amd import kaldo
    c3, ph3, g3, T, sigma = _sige648()
    c4 = sige_supercell(reps=4)
    _say("case: gamma interpolation 648 -> 1536 modes, oracle side")
    ph4 = P.phonons(c4, velocities=False)
    w_src, g_src = ph3.omega[0], g3[:, 0, :]
    nb = 48
    gi_ref = I.interpolate_gamma(w_src, g_src, ph4.omega[0], ph4.sets[0], nb)[:, None, :]
    k_ref = C.kappa_qhgk(c4, ph4, gi_ref, T)
    _say("case: gamma interpolation 648 -> 1536 modes, GPU")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c4)
        gi = ctx.gamma_interpolate(w_src, g_src, n_bins=nb, T=T)
        k = ctx.kappa_qhgk()
        # the same source from device memory: the same bits
        dw, dg = DeviceArray(w_src.shape, w_src), DeviceArray(g_src.shape, g_src)
        try:
            gi_dev = ctx.gamma_interpolate(dw, dg, n_bins=nb, T=T)
        finally:
            dw.free()
            dg.free()
    eg, ek = gamma_error(gi, gi_ref, ph4.mask[0]), kappa_error(k, k_ref)
    _say(f"  gamma error {eg:.3e}, kappa error {ek:.3e}")
    assert eg < 1e-10, eg
    assert ek < 1e-10, ek
    assert np.array_equal(gi, gi_dev)


def test_new_calls_reject_bad_input():
    from paper_2009_01967_amd import kaldo
    c = sige_supercell(reps=1)
    g = np.full((1, 1, c.n_modes), 0.1)
    with kaldo.Context(0) as ctx:
        assert kaldo.kaldo_set_gamma(ctx.h, [300.0], kaldo.KALDO_QUANTUM, g) == kaldo.KALDO_ESTATE
        w = np.linspace(1.0, 10.0, 5)
        assert kaldo.kaldo_gamma_interpolate(ctx.h, [300.0], 0, w, w[None], 5, 4) == kaldo.KALDO_ESTATE
        assert kaldo.kaldo_qhgk_options(ctx.h, -1.0, 0.0) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_qhgk_options(ctx.h, 0.0, float("nan")) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_qhgk_options(ctx.h, float("inf"), 0.0) == kaldo.KALDO_EINVAL
        ctx.phonons(c)
        bad = g.copy()
        bad[0, 0, 5] = -1.0
        assert kaldo.kaldo_set_gamma(ctx.h, [300.0], kaldo.KALDO_QUANTUM, bad) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_set_gamma(ctx.h, [], kaldo.KALDO_QUANTUM, g) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_gamma_interpolate(ctx.h, [300.0], 0, w, w[None], 5, 0) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_gamma_interpolate(ctx.h, [300.0], 0, w, w[None], 5, 5000) == kaldo.KALDO_EINVAL
        zero = np.zeros(5)
        assert kaldo.kaldo_gamma_interpolate(ctx.h, [300.0], 0, zero, w[None], 5, 4) == kaldo.KALDO_EINVAL
    d = diamond_si(grid=(3, 3, 3), rc3=2.6, seed=3)
    with kaldo.Context(0) as ctx:
        ctx.phonons(d)
        ctx.linewidths(d, T=[300.0], sigma_thz=0.2)
        ctx.set_gamma(T=[300.0], gamma=np.full((1, 27, 6), 0.1))
        out = np.zeros((1, 3, 3))
        assert kaldo.kaldo_kappa_bte(ctx.h, 0, 10, 1e-10, out) == kaldo.KALDO_ESTATE
        ctx.linewidths(d, T=[300.0], sigma_thz=0.2)
        kaldo._check(ctx.h, kaldo.kaldo_kappa_bte(ctx.h, 0, 10, 1e-10, out))
