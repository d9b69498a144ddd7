"""kaldo_kappa_rta_noalloc (no device allocation; partial sums in the
library's static scratch array) against kaldo_kappa_rta on the same context,
on two calls in a row, the second with a smaller input (fewer temperatures,
fewer modes), so that a value left in the scratch array by the first call
would show."""

import ctypes
import sys

import numpy as np
import pytest

from gen import diamond_si

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    ("diamond 5x5x5 shell 2, 3 T", dict(grid=(5, 5, 5), rc3=3.9, seed=11), [100.0, 300.0, 600.0]),
    ("diamond 3x3x3 shell 1, 1 T", dict(grid=(3, 3, 3), rc3=2.6, seed=12), [300.0]),
]


class DeviceArray:
    """Doubles in device memory from hipMalloc of the HIP runtime the library
    uses (torch's runtime cannot initialise the GPU once the library has used
    it in the process, which earlier test modules do)."""

    def __init__(self, shape):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.shape = shape
        self.nbytes = int(np.prod(shape)) * 8
        self.ptr = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(self.nbytes)) == 0

    def data_ptr(self):
        return self.ptr.value

    def numpy(self):
        out = np.empty(self.shape)
        assert self.hip.hipDeviceSynchronize() == 0
        assert self.hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), self.ptr, ctypes.c_size_t(self.nbytes), 2) == 0
        return out

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()


def test_noalloc_kappa_matches_kappa_rta_on_two_calls():
    from paper_2009_01967_amd import kaldo
    for name, kw, T in CASES:
        _say(f"case: kaldo_kappa_rta_noalloc, {name}")
        c = diamond_si(**kw)
        with kaldo.Context(0) as ctx:
            ctx.phonons(c)
            ctx.linewidths(c, T=T, sigma_thz=0.1, precision="fp64")
            got = np.full((len(T), 3, 3), np.nan)
            kaldo._check(ctx.h, kaldo.kaldo_kappa_rta_noalloc(ctx.h, got))
            ref = ctx.kappa_rta()
            assert np.array_equal(got, ref), (name, got, ref)
            dev = DeviceArray((len(T), 3, 3))
            try:
                kaldo._check(ctx.h, kaldo.kaldo_kappa_rta_noalloc(ctx.h, dev))
                assert np.array_equal(dev.numpy(), ref), name
            finally:
                dev.free()
        _say(f"  equal to kaldo_kappa_rta: {ref[0, 0, 0]:.6e} W/m/K")


def test_noalloc_kappa_errors():
    from paper_2009_01967_amd import kaldo
    c = diamond_si(grid=(2, 2, 2), rc3=2.6, seed=13)
    with kaldo.Context(0) as ctx:
        out = np.zeros((1, 3, 3))
        assert kaldo.kaldo_kappa_rta_noalloc(ctx.h, out) == kaldo.KALDO_ESTATE
        ctx.phonons(c)
        ctx.linewidths(c, T=[300.0], sigma_thz=0.1, precision="fp64")
        assert kaldo.kaldo_kappa_rta_noalloc(ctx.h, None) == kaldo.KALDO_EINVAL
