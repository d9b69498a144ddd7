"""Caller-provided device memory (kaldo_set_workspace): a context whose buffers
all come from one caller allocation gives the same linewidths and conductivity,
bit for bit, as one that allocates its own; a workspace that is too small fails
with KALDO_ENOMEM; misuse is rejected.  The caller's memory comes from hipMalloc
of the HIP runtime the library uses (torch would have to initialise the GPU
before the library's first call in the process, which other test modules
have already made)."""

import ctypes
import sys

import numpy as np
import pytest

from gen import workload, batch_crystals

pytestmark = pytest.mark.gpu

T = [300.0, 600.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class DeviceMemory:
    """hipMalloc'd bytes from the library's own HIP runtime."""

    def __init__(self, nbytes):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.ptr = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes)) == 0
        self.nbytes = nbytes

    def pair(self):
        return (self.ptr.value, self.nbytes)

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()


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
    mem = DeviceMemory(256 << 20)
    with kaldo.Context(0, workspace=mem.pair()) as ctx:
        g1, k1 = _run(ctx, c, precision)
    mem.free()
    assert np.array_equal(g0, g1)
    assert np.array_equal(k0, k1)


def test_workspace_batch():
    from paper_2009_01967_amd import kaldo
    crystals = batch_crystals(count=2, n_range=(2, 5), g_range=(3, 3))
    _say("case: batch in a workspace")
    res = []
    mem = DeviceMemory(512 << 20)
    for ws in (None, mem.pair()):
        with kaldo.Context(0, workspace=ws) as ctx:
            kaldo._check(ctx.h, kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_FIXED))
            for cr in crystals:
                ctx.batch_add(cr)
            res.append(ctx.batch_run(T=T, sigma_thz=0.3, precision="fp32"))
    mem.free()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_workspace_too_small_and_misuse():
    from paper_2009_01967_amd import kaldo
    c = workload("diamond-2at-4x4x4-shell1")
    _say("case: workspace errors")
    small = DeviceMemory(64 << 10)
    with kaldo.Context(0, workspace=small.pair()) as ctx:
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
        assert kaldo.kaldo_set_workspace(ctx.h, *small.pair()) == kaldo.KALDO_ESTATE
    small.free()
