"""Linewidth interpolation in frequency for large disordered cells (Sec. II.C:
gamma computed on a smaller cell is interpolated as a function of frequency
with third-order splines and used for the QHGK conductivity of the larger
cell; Sec. IV.B uses it from a 3x3x3 to a 5x5x5 replica).  Plain FP64 NumPy.
Test infrastructure: only tests/, the package smoke check and the benchmark's
CPU leg call it.

Readings of points the paper leaves open (it names only "third-order
splines"):
* gamma(omega) of a disordered cell scatters from mode to mode, and nearly
  equal frequencies carry different linewidths, so the spline does not pass
  through every mode: the unmasked source modes (nu >= 0.01 THz) are put into
  n_bins bins of equal width between their lowest and highest frequency, bin
  b = floor((w - w_lo) / (w_hi - w_lo) * n_bins) (the highest mode in the last
  bin), and each non-empty bin gives one knot: the mean frequency and the mean
  linewidth of its modes.
* The spline is the natural cubic spline through the knots (second
  derivative 0 at both ends): one knot gives a constant, two a straight line.
* Outside the first and last knot the end knot's linewidth is kept; the
  spline is bounded below by the smallest knot linewidth (an interpolant of
  positive linewidths that dips below them is not a linewidth).
* Target modes that are masked get 0; within a degenerate set of the target
  the interpolated values are averaged, as computed linewidths are.
"""

from __future__ import annotations

import numpy as np

from . import units


def frequency_knots(omega, gamma, mask, n_bins):
    """Knots (x, y) of the binned means: omega, gamma, mask flat arrays of the
    source modes [rad/ps]; returns knot frequencies (ascending) and linewidths."""
    w = np.asarray(omega, dtype=float)[mask]
    g = np.asarray(gamma, dtype=float)[mask]
    if w.size == 0:
        raise ValueError("no unmasked source modes")
    lo, hi = w.min(), w.max()
    if hi > lo:
        b = np.floor((w - lo) / (hi - lo) * n_bins).astype(np.int64)
        b = np.minimum(b, n_bins - 1)
    else:
        b = np.zeros(w.size, dtype=np.int64)
    xs, ys = [], []
    for k in range(n_bins):
        sel = b == k
        if np.any(sel):
            xs.append(np.sum(w[sel]) / np.count_nonzero(sel))
            ys.append(np.sum(g[sel]) / np.count_nonzero(sel))
    return np.array(xs), np.array(ys)


def natural_spline_second_derivatives(x, y):
    """M_i = s''(x_i) of the natural cubic spline through (x_i, y_i): the
    continuity of s' at the interior knots,
      h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
          = 6 ((y_{i+1} - y_i)/h_i - (y_i - y_{i-1})/h_{i-1}),
    with M_0 = M_{m-1} = 0 (solved as one dense system)."""
    m = len(x)
    M = np.zeros(m)
    if m < 3:
        return M
    h = np.diff(x)
    A = np.zeros((m - 2, m - 2))
    r = np.zeros(m - 2)
    for i in range(1, m - 1):
        j = i - 1
        A[j, j] = 2.0 * (h[i - 1] + h[i])
        if j > 0:
            A[j, j - 1] = h[i - 1]
        if j < m - 3:
            A[j, j + 1] = h[i]
        r[j] = 6.0 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1])
    M[1:-1] = np.linalg.solve(A, r)
    return M


def spline_eval(x, y, M, t):
    """The cubic on the knot interval [x_i, x_{i+1}] holding t, in the form
      s = (M_i (x_{i+1} - t)^3 + M_{i+1} (t - x_i)^3) / (6 h)
          + (y_i - M_i h^2 / 6) (x_{i+1} - t) / h + (y_{i+1} - M_{i+1} h^2 / 6) (t - x_i) / h,
    the end values outside [x_0, x_{m-1}]."""
    t = np.asarray(t, dtype=float)
    m = len(x)
    if m == 1:
        return np.full(t.shape, y[0])
    out = np.empty(t.shape)
    for idx, tv in np.ndenumerate(t):
        if tv <= x[0]:
            out[idx] = y[0]
            continue
        if tv >= x[-1]:
            out[idx] = y[-1]
            continue
        i = int(np.searchsorted(x, tv, side='right')) - 1
        h = x[i + 1] - x[i]
        a, b = x[i + 1] - tv, tv - x[i]
        out[idx] = ((M[i] * a ** 3 + M[i + 1] * b ** 3) / (6.0 * h)
                    + (y[i] - M[i] * h * h / 6.0) * a / h + (y[i + 1] - M[i + 1] * h * h / 6.0) * b / h)
    return out


def interpolate_gamma(omega_src, gamma_src, omega_dst, sets_dst, n_bins):
    """gamma on the target modes from the source modes' gamma(omega).
    omega_src: flat source frequencies [rad/ps]; gamma_src: (nT, len(omega_src))
    [rad/ps]; omega_dst: target frequencies; sets_dst: the target's degenerate
    sets (index arrays).  Returns (nT, len(omega_dst))."""
    omega_src = np.asarray(omega_src, dtype=float)
    omega_dst = np.asarray(omega_dst, dtype=float)
    gamma_src = np.atleast_2d(np.asarray(gamma_src, dtype=float))
    mask_src = omega_src / units.TWO_PI >= units.NU_MIN_THZ
    mask_dst = omega_dst / units.TWO_PI >= units.NU_MIN_THZ
    out = np.zeros((gamma_src.shape[0], omega_dst.size))
    for it in range(gamma_src.shape[0]):
        x, y = frequency_knots(omega_src, gamma_src[it], mask_src, n_bins)
        M = natural_spline_second_derivatives(x, y)
        g = np.maximum(spline_eval(x, y, M, omega_dst), y.min())
        g = np.where(mask_dst, g, 0.0)
        for S in sets_dst:
            g[S] = g[S].mean()
        out[it] = g
    return out
