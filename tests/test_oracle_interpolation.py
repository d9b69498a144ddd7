"""Pins of the oracle's linewidth interpolation in frequency (Sec. II.C and
Sec. IV.B: third-order splines from a smaller cell): a natural cubic spline
worked by hand, scipy's natural spline as an independent library routine,
continuity of the first and second derivatives, exact reproduction of a
straight line through the whole binned pipeline, the binning brute-forced on
a small input, and the end, floor, mask and degenerate-set rules."""

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import interpolation as I, units


def test_hand_worked_natural_spline():
    """Knots (0, 0), (1, 1), (2, 0): the one interior equation is
    2 (1 + 1) M_1 = 6 ((0 - 1) - (1 - 0)), so M_1 = -3, and at t = 1/2
    s = (-3 / 8) / 6 + (1 + 3 / 6) / 2 = 0.6875."""
    x, y = np.array([0.0, 1.0, 2.0]), np.array([0.0, 1.0, 0.0])
    M = I.natural_spline_second_derivatives(x, y)
    assert np.allclose(M, [0.0, -3.0, 0.0], atol=1e-15)
    assert I.spline_eval(x, y, M, np.array([0.5]))[0] == pytest.approx(0.6875, rel=1e-15)
    assert I.spline_eval(x, y, M, np.array([1.5]))[0] == pytest.approx(0.6875, rel=1e-15)


def test_spline_matches_scipy_natural_spline():
    rng = np.random.default_rng(3)
    x = np.cumsum(rng.uniform(0.1, 2.0, 23))
    y = rng.uniform(0.1, 3.0, 23)
    M = I.natural_spline_second_derivatives(x, y)
    t = np.linspace(x[0], x[-1], 1001)
    ref = CubicSpline(x, y, bc_type="natural")
    assert np.allclose(I.spline_eval(x, y, M, t), ref(t), rtol=1e-12, atol=1e-12)
    assert np.allclose(M, ref(x, 2), rtol=1e-10, atol=1e-10)


def test_spline_passes_the_knots_with_continuous_derivatives():
    rng = np.random.default_rng(4)
    x = np.cumsum(rng.uniform(0.2, 1.0, 9))
    y = rng.uniform(-1.0, 1.0, 9)
    M = I.natural_spline_second_derivatives(x, y)
    assert np.allclose(I.spline_eval(x, y, M, x), y, rtol=1e-14, atol=1e-14)
    h = 1e-5
    for xi in x[1:-1]:
        l1 = (I.spline_eval(x, y, M, [xi])[0] - I.spline_eval(x, y, M, [xi - h])[0]) / h
        r1 = (I.spline_eval(x, y, M, [xi + h])[0] - I.spline_eval(x, y, M, [xi])[0]) / h
        assert l1 == pytest.approx(r1, abs=1e-3)
        s = I.spline_eval(x, y, M, [xi - 2 * h, xi - h, xi, xi + h, xi + 2 * h])
        l2 = (s[2] - 2 * s[1] + s[0]) / h ** 2
        r2 = (s[4] - 2 * s[3] + s[2]) / h ** 2
        assert l2 == pytest.approx(r2, abs=2e-2 * (1 + abs(l2)))
    # natural ends: zero curvature at the first and last knot
    s = I.spline_eval(x, y, M, [x[0], x[0] + h, x[0] + 2 * h])
    assert abs((s[2] - 2 * s[1] + s[0]) / h ** 2) < 2e-2 * (1 + np.abs(M).max())


def test_binning_brute_force():
    """Each source mode in bin floor((w - lo) / (hi - lo) * nb), the highest in
    the last bin, masked modes left out; knots are the bins' mean w and gamma."""
    rng = np.random.default_rng(5)
    w = rng.uniform(0.0, 40.0, 200)
    w[:3] = [0.0, 0.01, 0.02]                             # below 0.01 THz: masked
    g = rng.uniform(0.1, 2.0, 200)
    mask = w / units.TWO_PI >= units.NU_MIN_THZ
    nb = 7
    x, y = I.frequency_knots(w, g, mask, nb)
    lo, hi = w[mask].min(), w[mask].max()
    xs, ys = [], []
    for b in range(nb):
        members = []
        for i in range(w.size):
            if not mask[i]:
                continue
            bi = int((w[i] - lo) / (hi - lo) * nb)
            if bi == nb:
                bi = nb - 1
            if bi == b:
                members.append(i)
        if members:
            xs.append(sum(w[i] for i in members) / len(members))
            ys.append(sum(g[i] for i in members) / len(members))
    assert np.allclose(x, xs, rtol=1e-14) and np.allclose(y, ys, rtol=1e-14)
    assert np.all(np.diff(x) > 0)


def test_straight_line_is_reproduced_through_the_bins():
    """gamma = a + b w on the source: each bin's mean (w, gamma) lies on the
    line, the natural spline through points on a line is the line, so the
    target gets a + b w exactly inside the knot range and the end values
    outside it."""
    rng = np.random.default_rng(6)
    a, b = 0.3, 0.02
    ws = rng.uniform(1.0, 60.0, 3000)
    gs = a + b * ws
    wd = np.concatenate((rng.uniform(5.0, 55.0, 400), [0.5, 70.0, 0.03]))
    sets = [np.array([i]) for i in range(wd.size)]
    out = I.interpolate_gamma(ws, gs[None], wd, sets, 40)[0]
    x, y = I.frequency_knots(ws, gs, ws / units.TWO_PI >= units.NU_MIN_THZ, 40)
    inside = (wd >= x[0]) & (wd <= x[-1])
    assert np.allclose(out[inside], a + b * wd[inside], rtol=1e-12)
    assert out[-3] == pytest.approx(y[0], rel=1e-14)      # below the first knot
    assert out[-2] == pytest.approx(y[-1], rel=1e-14)     # above the last knot
    assert out[-1] == 0.0                                 # masked target mode


def test_constant_floor_and_degenerate_sets():
    ws = np.linspace(1.0, 10.0, 50)
    out = I.interpolate_gamma(ws, np.full((2, 50), 0.7), np.array([2.0, 3.0]), [np.array([0]), np.array([1])], 8)
    assert np.allclose(out, 0.7, rtol=1e-14)
    # a spike: the natural spline undershoots beside it; the floor is the smallest knot
    ws = np.arange(1.0, 11.0)
    gs = np.full(10, 0.1)
    gs[5] = 5.0
    x, y = I.frequency_knots(ws, gs, np.ones(10, bool), 10)
    M = I.natural_spline_second_derivatives(x, y)
    t = np.linspace(1.0, 10.0, 901)
    assert I.spline_eval(x, y, M, t).min() < 0.1          # the raw spline dips below
    out = I.interpolate_gamma(ws, gs[None], t, [np.array([i]) for i in range(t.size)], 10)[0]
    assert out.min() == pytest.approx(0.1, rel=1e-14)
    # a degenerate target set gets the mean of its members' values
    wd = np.array([3.2, 3.2 + 1e-9, 6.1])
    raw = I.interpolate_gamma(ws, gs[None], wd, [np.array([0]), np.array([1]), np.array([2])], 10)[0]
    avg = I.interpolate_gamma(ws, gs[None], wd, [np.array([0, 1]), np.array([2])], 10)[0]
    assert avg[0] == avg[1] == pytest.approx(0.5 * (raw[0] + raw[1]), rel=1e-14)
    assert avg[2] == raw[2]
