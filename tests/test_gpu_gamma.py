"""Gamma-point path (grid {1,1,1}) through the C ABI against the FP64 oracle:
linewidths of disordered and folded cells in FP64, FP32 and BF16X3, and the
QHGK conductivity."""

import sys

import numpy as np
import pytest

from gen import diamond_si, sige_supercell, WORKLOADS
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A, conductivity as C
from tests.parity import TOL, gamma_error, kappa_error
from tests.supercell import fold

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ok(err, tol):
    print(f"  error {err:.3e} (tolerance {tol:.0e})", flush=True)
    assert err < tol, err


def _ctx():
    from paper_2009_01967_amd import kaldo
    return kaldo.Context(0)


@pytest.fixture(scope="module")
def folded_diamond():
    # 16-atom folded crystal: 48 modes (one partial 64-tile), degenerate sets
    c = fold(diamond_si(grid=(2, 2, 2), rc3=4.0, masses=(M_SI, M_GE), seed=17))
    ph = P.phonons(c, velocities=False)
    g = A.linewidths(c, ph, [100.0, 300.0], 0.3)
    return c, ph, g


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_folded_crystal_gamma_point(folded_diamond, precision):
    c, ph, g = folded_diamond
    _say(f"case: folded diamond 16 atoms at Gamma, {precision}")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=[100.0, 300.0], sigma_thz=0.3, precision=precision)
    _ok(gamma_error(gg, g, ph.mask), TOL[precision])


@pytest.fixture(scope="module")
def sige64():
    name = "sige-64at-gamma"
    w = WORKLOADS[name]
    c = sige_supercell(reps=2, rc3=4.0)
    ph = P.phonons(c, velocities=False)
    g = A.linewidths_gamma_sparse(c, ph, w["T"], w["sigma_thz"])[:, None, :]
    k = C.kappa_qhgk(c, ph, g, w["T"])
    return c, w, ph, g, k


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_disordered_sige64_linewidths_and_qhgk(sige64, precision):
    c, w, ph, g, k = sige64
    _say(f"case: sige 64 atoms at Gamma, {precision}")
    with _ctx() as ctx:
        nu = ctx.phonons(c)
        gg = ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision=precision)
        kq = ctx.kappa_qhgk()
    lam = np.sign(nu) * nu ** 2
    lam_ref = np.sign(ph.nu) * ph.nu ** 2
    assert np.max(np.abs(lam - lam_ref)) < 1e-11 * np.abs(lam_ref).max()
    _ok(gamma_error(gg, g, ph.mask), TOL[precision])
    _ok(kappa_error(kq, k), TOL[precision])


def test_qhgk_several_temperatures_and_classical(sige64):
    c, w, ph, _, _ = sige64
    T = [50.0, 300.0, 900.0]
    _say("case: sige 64 QHGK, 3 temperatures, quantum and classical")
    for stats in ("quantum", "classical"):
        g = A.linewidths_gamma_sparse(c, ph, T, 0.2, stats=stats)[:, None, :]
        k = C.kappa_qhgk(c, ph, g, T, stats=stats)
        with _ctx() as ctx:
            ctx.phonons(c)
            gg = ctx.linewidths(c, T=T, sigma_thz=0.2, classical=stats == "classical")
            kq = ctx.kappa_qhgk()
        _ok(gamma_error(gg, g, ph.mask), TOL["fp64"])
        _ok(kappa_error(kq, k), TOL["fp64"])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_full_size_sige_1000_atoms_sampled_modes(precision):
    """1000-atom disordered SiGe (3000 modes) at full size; the oracle
    evaluates sampled first modes one by one."""
    name = "sige-1000at-gamma"
    w = WORKLOADS[name]
    _say(f"case: {name} {precision}: generating")
    c = sige_supercell(reps=5, rc3=4.0)
    _say("  GPU run")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision=precision)
    _say("  oracle eigensolve")
    ph = P.phonons(c, velocities=False)
    ss = [3, 4, 777, 1500, 2998, 2999]
    cols = []
    for s in ss:
        _say(f"  oracle mode {s}")
        cols.append(A.linewidths_gamma_sparse(c, ph, w["T"], w["sigma_thz"], s_subset=[s]))
    g = np.concatenate(cols, axis=1)
    _ok(gamma_error(gg[:, 0, ss], g, ph.mask[0, ss]), TOL[precision])
    assert np.all(gg[:, 0, :3] == 0.0)
