"""Many-branch crystal path (two chained complex MFMA GEMMs with the fused
epilogue) through the C ABI against the FP64 oracle."""

import sys

import numpy as np
import pytest

from gen import diamond_si, random_crystal, cage_cell, WORKLOADS
from gen.crystals import M_SI, M_GE
from oracle import phonons as P, anharmonic as A
from tests.parity import TOL, gamma_error, kappa_error, oracle_all

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


@pytest.mark.parametrize("n_atoms", [11, 22])
def test_library_eigensolver_sizes(n_atoms):
    """Beyond the LDS Jacobi range (n > 32, and n > 64) the batched library
    eigensolver is used: its eigenvectors must give finite, correct velocities."""
    rng = np.random.default_rng(5)
    c = random_crystal(n_atoms, 2, rng).with_grid((3, 2, 1))
    _say(f"case: eigensolver, {c.n_modes} branches")
    ph = P.phonons(c)
    with _ctx() as ctx:
        vel = np.zeros((c.n_k, c.n_modes, 3))
        nu = ctx.phonons(c, vel_out=vel)
    assert np.all(np.isfinite(vel))
    lam = np.sign(nu) * nu ** 2
    lam_ref = np.sign(ph.nu) * ph.nu ** 2
    assert np.max(np.abs(lam - lam_ref)) < 1e-11 * np.abs(lam_ref).max()
    for k in range(c.n_k):
        for S in ph.sets[k]:
            if len(S) == 1 and ph.mask[k, S[0]]:
                d = float(np.abs(vel[k, S[0]] - ph.velocity[k, S[0]]).max())
                assert d < 1e-9 * max(1.0, np.abs(ph.velocity).max()), (k, S[0], d)


@pytest.fixture(scope="module")
def four_atom():
    # 12 branches, grid 3x3x2 (18 points), Si/Ge species, pair-spring fc2
    rng = np.random.default_rng(404)
    c = random_crystal(4, 3, rng).with_grid((3, 3, 2))
    T = [150.0, 600.0]
    ph, g, k = oracle_all(c, T, 0.3)
    return c, T, ph, g, k


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_four_atom_crystal(four_atom, precision):
    c, T, ph, g, k = four_atom
    _say(f"case: 4-atom crystal 3x3x2, {precision}")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=T, sigma_thz=0.3, precision=precision)
        kk = ctx.kappa_rta()
    _ok(gamma_error(gg, g, ph.mask), TOL[precision])
    _ok(kappa_error(kk, k), TOL[precision])


def test_two_atom_diamond_bf16x3():
    w = WORKLOADS["diamond-2at-4x4x4-shell1"]
    c = diamond_si(grid=(4, 4, 4), rc3=2.6)
    _say("case: diamond 4x4x4 bf16x3 (many-branch path at n = 6)")
    ph, g, k = oracle_all(c, w["T"], w["sigma_thz"])
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision="bf16x3")
        kk = ctx.kappa_rta()
    _ok(gamma_error(gg, g, ph.mask), TOL["bf16x3"])
    _ok(kappa_error(kk, k), TOL["bf16x3"])


@pytest.fixture(scope="module")
def cage_reference():
    name = "cage-46at-5x5x5"
    w = WORKLOADS[name]
    _say(f"oracle: {name}: generating")
    c = cage_cell(grid=w["grid"], rc3=w["rc3"])
    ph = P.phonons(c, velocities=False)
    ks = [0, 7, 62]
    cols = []
    for k in ks:
        _say(f"  oracle k = {k}")
        cols.append(A.linewidths(c, ph, w["T"], w["sigma_thz"], k_subset=[k]))
    return c, w, ph, ks, np.concatenate(cols, axis=1)


@pytest.mark.parametrize("precision", ["bf16x3", "fp32", "fp64"])
def test_full_size_cage_46_atoms_sampled_k(cage_reference, precision):
    """46-atom cage cell (138 branches) on 5x5x5 at full size; the oracle
    evaluates sampled first-mode k points (0; 7 = (0,1,2); 62 = (2,2,2)).  The
    GPU computes one point of each pair (k, -k) and stores it at both: the
    mirrors 23 = (0,4,3) and 93 = (3,3,3) must hold the same values."""
    c, w, ph, ks, g = cage_reference
    _say(f"case: cage-46at-5x5x5 {precision}")
    with _ctx() as ctx:
        ctx.phonons(c)
        gg = ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision=precision)
    _ok(gamma_error(gg[:, ks], g, ph.mask[ks]), TOL[precision])
    assert np.array_equal(gg[:, 23], gg[:, 7]) and np.array_equal(gg[:, 93], gg[:, 62])
