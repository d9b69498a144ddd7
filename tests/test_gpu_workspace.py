"""Caller-provided device memory (kaldo_set_workspace): a context whose buffers
all come from one torch allocation gives the same linewidths and conductivity,
bit for bit, as one that allocates its own; a workspace that is too small fails
with KALDO_ENOMEM; misuse is rejected."""

import sys

import numpy as np
import pytest

from gen import workload, batch_crystals

pytestmark = pytest.mark.gpu

T = [300.0, 600.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(ctx, c, precision):
    from paper_2009_01967_amd import kaldo
    kaldo._check(ctx.h, kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_FIXED))
    ctx.phonons(c)
    g = ctx.linewidths(c, T=T, sigma_thz=0.2, precision=precision)
    return g, ctx.kappa_rta()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_workspace_results_equal_own_allocations(precision):
    from paper_2009_01967_amd import kaldo
    c = workload("diamond-2at-4x4x4-shell1")
    _say(f"case: workspace vs own allocations, diamond 4x4x4, {precision}")
    with kaldo.Context(0) as ctx:
        g0, k0 = _run(ctx, c, precision)
    with kaldo.Context(0, workspace_bytes=256 << 20) as ctx:
        g1, k1 = _run(ctx, c, precision)
    assert np.array_equal(g0, g1)
    assert np.array_equal(k0, k1)


def test_workspace_batch():
    from paper_2009_01967_amd import kaldo
    crystals = batch_crystals(count=2, n_range=(2, 5), g_range=(3, 3))
    _say("case: batch in a workspace")
    res = []
    for ws in (None, 512 << 20):
        with kaldo.Context(0, workspace_bytes=ws) as ctx:
            kaldo._check(ctx.h, kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_FIXED))
            for cr in crystals:
                ctx.batch_add(cr)
            res.append(ctx.batch_run(T=T, sigma_thz=0.3, precision="fp32"))
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_workspace_too_small_and_misuse():
    import torch
    from paper_2009_01967_amd import kaldo
    c = workload("diamond-2at-4x4x4-shell1")
    _say("case: workspace errors")
    with kaldo.Context(0, workspace_bytes=64 << 10) as ctx:
        keep = kaldo._Keep()
        s = kaldo.make_structure(c.cell, c.positions, c.masses, keep)
        f2 = kaldo.make_fc2(c.fc2_i, c.fc2_j, c.fc2_R, c.fc2_val, keep)
        st = kaldo.kaldo_phonons(ctx.h, s, f2, c.grid, None, None)
        assert st == kaldo.KALDO_ENOMEM
        assert "short" in kaldo.kaldo_last_error(ctx.h)
    with kaldo.Context(0) as ctx:
        host = np.zeros(1 << 16, np.uint8)
        assert kaldo.kaldo_set_workspace(ctx.h, host.ctypes.data, host.nbytes) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_set_workspace(ctx.h, None, 16) == kaldo.KALDO_EINVAL
        ctx.phonons(c)
        buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
        assert kaldo.kaldo_set_workspace(ctx.h, buf.data_ptr(), buf.numel()) == kaldo.KALDO_ESTATE
