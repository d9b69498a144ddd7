"""Device arrays for GPU tests from hipMalloc of the HIP runtime the library
uses (torch's runtime cannot initialise the GPU once the library has used it
in the process, which earlier test modules do)."""

import ctypes

import numpy as np


class DeviceArray:
    """Doubles in device memory; ``data_ptr()`` is what the bindings pass on."""

    def __init__(self, shape, host=None):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.shape = tuple(shape)
        self.nbytes = int(np.prod(self.shape)) * 8
        self.ptr = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(self.nbytes)) == 0
        if host is not None:
            h = np.ascontiguousarray(host, dtype=np.float64).reshape(self.shape)
            assert self.hip.hipMemcpy(self.ptr, ctypes.c_void_p(h.ctypes.data), ctypes.c_size_t(self.nbytes), 1) == 0

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
