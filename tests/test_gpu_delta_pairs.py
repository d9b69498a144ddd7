"""Step B of the few-branch kernel sums each (Delta, -Delta) pair of
Delta = R2 - R1 through the sum and difference of its two A_k slots, and every
Delta without its negative (and Delta = 0) on its own.  Here the diamond 4x4x4
constants lose every block with one chosen Delta, which leaves -Delta unpaired,
and the GPU linewidths (FP32, which uses the pairs, and FP64) are compared with
the FP64 oracle on the same constants.  The oracle sums over the blocks as
given, so the missing permutation partners change nothing in its definition."""

import dataclasses
import sys

import numpy as np
import pytest

from gen import workload
from oracle import phonons as P, anharmonic as A
from tests.parity import TOL, gamma_error

pytestmark = pytest.mark.gpu

T = [300.0]
SIGMA = 0.25


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def unpaired():
    c = workload("diamond-2at-4x4x4-shell1")
    d = c.fc3_R2 - c.fc3_R1
    dset = {tuple(int(v) for v in x) for x in d}
    pos = sorted(x for x in dset if x > (0, 0, 0) and tuple(-v for v in x) in dset)
    assert len(pos) >= 2, "the shell has (Delta, -Delta) pairs"
    drop = np.array(pos[0])
    keep = np.any(d != drop, axis=1)
    c2 = dataclasses.replace(c, fc3_i=c.fc3_i[keep], fc3_j=c.fc3_j[keep], fc3_l=c.fc3_l[keep],
                             fc3_R1=c.fc3_R1[keep], fc3_R2=c.fc3_R2[keep], fc3_val=c.fc3_val[keep])
    d2 = {tuple(int(v) for v in x) for x in (c2.fc3_R2 - c2.fc3_R1)}
    assert pos[0] not in d2 and tuple(-v for v in pos[0]) in d2
    _say(f"oracle: diamond 4x4x4 without Delta = {pos[0]} ({int((~keep).sum())} blocks dropped)")
    ph = P.phonons(c2, velocities=False)
    g = A.linewidths(c2, ph, T, SIGMA)
    return c2, ph, g


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_unpaired_delta_against_oracle(unpaired, precision):
    from paper_2009_01967_amd import kaldo
    c, ph, g_ref = unpaired
    _say(f"case: diamond 4x4x4 with an unpaired Delta, {precision}")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        g = ctx.linewidths(c, T=T, sigma_thz=SIGMA, precision=precision)
    err = gamma_error(g, g_ref, ph.mask)
    _say(f"  error {err:.3e} (tolerance {TOL[precision]:.0e})")
    assert err < TOL[precision], err
