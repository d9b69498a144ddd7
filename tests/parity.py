"""Shared helpers for GPU-vs-oracle parity tests: error metrics and oracle runs."""

import numpy as np

from oracle import phonons as P, anharmonic as A, conductivity as C

# Tolerances by projection precision (relative, gamma and kappa).
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}


def gamma_error(g, g_ref, mask):
    """max over unmasked modes of |g - g_ref| / max(g_ref, 1e-6 max g_ref)."""
    g = np.asarray(g)
    g_ref = np.asarray(g_ref)
    m = np.broadcast_to(mask, g_ref.shape)
    ref = np.abs(g_ref[m])
    floor = 1e-6 * ref.max() if ref.size else 0.0
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(g[m] - g_ref[m]) / np.maximum(ref, floor)))


def kappa_error(k, k_ref):
    return float(np.linalg.norm(np.asarray(k) - k_ref) / np.linalg.norm(k_ref))


def set_average(ph, g, ks):
    """Average a (nT, len(ks), n) array over the oracle's degenerate sets."""
    out = g.copy()
    for ik, k in enumerate(ks):
        for S in ph.sets[k]:
            out[:, ik, S] = np.mean(g[:, ik, S], axis=-1, keepdims=True)
    return out


def oracle_all(crystal, T, sigma, stats="quantum", k_subset=None, kappa=True):
    ph = P.phonons(crystal, velocities=crystal.n_k > 1)
    g = A.linewidths(crystal, ph, T, sigma, stats=stats, k_subset=k_subset)
    k = None
    if kappa and k_subset is None:
        if crystal.n_k > 1:
            k = C.kappa_rta(crystal, ph, g, T, stats=stats)
        else:
            k = C.kappa_qhgk(crystal, ph, g, T, stats=stats)
    return ph, g, k
