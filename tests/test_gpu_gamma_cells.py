"""Gamma-point path on small and densely paired random cells against the FP64
oracle: 3, 5 and 7 atoms (fewer atoms than one block of the sparse step covers,
odd counts) and a 40-atom cell in which every atom pairs with all 40 (more
pairs per atom than the sparse step stages through registers), the latter with
each block width of the sparse step and each GEMM tile shape forced."""

import sys

import numpy as np
import pytest

from gen import random_crystal
from oracle import phonons as P, anharmonic as A
from tests.parity import TOL, gamma_error

pytestmark = pytest.mark.gpu

T = [150.0, 500.0]
SIGMA = 0.25
CELLS = {"3at": (3, 4.0), "5at": (5, 4.0), "7at": (7, 4.0), "40at-dense": (40, 6.5)}
_REF = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _reference(name):
    if name not in _REF:
        n, rc = CELLS[name]
        c = random_crystal(n, 1, np.random.default_rng(900 + n), rc=rc).with_grid((1, 1, 1))
        ph = P.phonons(c, velocities=False)
        g = A.linewidths_gamma_sparse(c, ph, T, SIGMA)[:, None, :]
        _REF[name] = (c, ph, g)
    return _REF[name]


def _run(c, precision, tuning=None):
    from paper_2009_01967_amd import kaldo
    with kaldo.Context(0) as ctx:
        if tuning is not None:
            kaldo._check(ctx.h, kaldo.kaldo_set_tuning(ctx.h, tuning))
        ctx.phonons(c)
        return ctx.linewidths(c, T=T, sigma_thz=SIGMA, precision=precision)


@pytest.mark.parametrize("name", ["3at", "5at", "7at"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_small_cells(name, precision):
    c, ph, g = _reference(name)
    _say(f"case: random {name} at Gamma, {precision}")
    gg = _run(c, precision)
    err = gamma_error(gg, g, ph.mask)
    _say(f"  error {err:.3e}")
    assert err < TOL[precision], err


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("v", [0, 1, 2])
def test_dense_cell_every_block_width(precision, v):
    from paper_2009_01967_amd import kaldo
    c, ph, g = _reference("40at-dense")
    _say(f"case: random 40at-dense at Gamma, {precision}, forced candidate {v}")
    gg = _run(c, precision, kaldo.KALDO_TUNE_SHAPE0 + v)
    err = gamma_error(gg, g, ph.mask)
    _say(f"  error {err:.3e}")
    assert err < TOL[precision], err
