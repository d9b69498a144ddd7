"""Matrix-core flop tally of the projection GEMMs (kaldo_profile_flops) and the
tile skip it exposes: with timing on, the linewidths are bitwise those of an
untimed run; a kernel with no cut (Lorentzian) runs every tile; at the full
1000-atom SiGe size at Gamma the Gaussian window skips tiles.  Outputs of a
skipped tile are checked against the oracle by the sampled full-size tests."""

import sys

import numpy as np
import pytest

from gen import diamond_si, random_crystal, workload, WORKLOADS
from gen.crystals import M_SI, M_GE
from tests.supercell import fold

pytestmark = pytest.mark.gpu

T = [300.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(c, precision, sigma, delta, timed):
    from paper_2009_01967_amd import kaldo
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.linewidths(c, T=T, sigma_thz=sigma, precision=precision, delta=delta)   # plans and tunes
        kaldo.kaldo_profile_enable(ctx.h, timed)
        g = ctx.linewidths(None, T=T, sigma_thz=sigma, precision=precision, delta=delta)
        ex, dense = kaldo.kaldo_profile_flops(ctx.h)
        kaldo.kaldo_profile_enable(ctx.h, False)
        assert kaldo.kaldo_profile_flops(ctx.h) == (0.0, 0.0)
    return g, ex, dense


CASES = {
    "four-atom-3x3x2": (lambda: random_crystal(4, 3, np.random.default_rng(404)).with_grid((3, 3, 2)), 0.3),
    "folded-16at-gamma": (lambda: fold(diamond_si(grid=(2, 2, 2), rc3=4.0, masses=(M_SI, M_GE), seed=17)), 0.3),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
@pytest.mark.parametrize("delta", ["gauss", "lorentz"])
def test_timed_run_is_identical_and_counted(name, precision, delta):
    build, sigma = CASES[name]
    c = build()
    _say(f"case: tally {name} {precision} {delta}")
    g0, ex0, dn0 = _run(c, precision, sigma, delta, False)
    g1, ex1, dn1 = _run(c, precision, sigma, delta, True)
    assert np.array_equal(g0, g1)
    assert ex0 == 0.0 and dn0 == 0.0
    _say(f"  executed {ex1:.3e} of {dn1:.3e} flops")
    assert 0.0 < ex1 <= dn1
    if delta == "lorentz":
        assert ex1 == dn1


def test_sige_1000_gaussian_window_skips_tiles():
    from paper_2009_01967_amd import kaldo
    name = "sige-1000at-gamma"
    w = WORKLOADS[name]
    _say(f"case: tally {name} bf16x3")
    c = workload(name)
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        ctx.linewidths(c, T=w["T"], sigma_thz=w["sigma_thz"], precision="bf16x3")
        kaldo.kaldo_profile_enable(ctx.h, True)
        ctx.linewidths(None, T=w["T"], sigma_thz=w["sigma_thz"], precision="bf16x3")
        ex, dense = kaldo.kaldo_profile_flops(ctx.h)
    n = c.n_modes
    _say(f"  executed {ex:.3e} of {dense:.3e} flops ({1 - ex / dense:.2%} skipped)")
    # every tile launched covers at least the 3 x 2 n^4 bf16 flops of the dense projection
    assert dense >= 3 * 2.0 * n ** 4
    assert 0.0 < ex < dense


@pytest.mark.parametrize("name", ["four-atom-3x3x2", "cage-12at", "folded-16at-gamma"])
def test_frequencies_ascend_at_every_grid_point(name):
    """The tile skip bounds a tile's frequencies by its first and last modes."""
    from paper_2009_01967_amd import kaldo
    from gen.crystals import cage_cell
    if name == "cage-12at":
        c = cage_cell(n_atoms=12, L=6.0, grid=(2, 2, 2))   # 36 modes: the library solver, not Jacobi
    else:
        c = CASES[name][0]()
    _say(f"case: ascending frequencies, {name} ({c.n_modes} modes, grid {c.grid})")
    with kaldo.Context(0) as ctx:
        nu = ctx.phonons(c)
    assert np.all(np.diff(nu, axis=1) >= 0.0)
