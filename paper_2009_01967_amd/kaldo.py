"""Python binding of ``libkaldo.so`` (argument marshalling only).

Every function of the C ABI in ``include/kaldo.h`` is exposed under the same
name; the ``Context`` class bundles them for numpy inputs and numpy or torch
outputs.  All arithmetic runs in the library's HIP kernels; this module never
computes results itself, and it raises if the library is missing.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkaldo.so")

KALDO_OK = 0
KALDO_EINVAL = -1
KALDO_ENOMEM = -2
KALDO_EDEVICE = -3
KALDO_ESTATE = -4
KALDO_EUNSTABLE = -5
KALDO_ENOCONV = -6
KALDO_BTE_INVERSE = 0
KALDO_BTE_SELF_CONSISTENT = 1
BTE_METHODS = {"inverse": KALDO_BTE_INVERSE, "self-consistent": KALDO_BTE_SELF_CONSISTENT}

KALDO_FP64 = 0
KALDO_FP32 = 1
KALDO_BF16X3 = 2
PRECISIONS = {"fp64": KALDO_FP64, "fp32": KALDO_FP32, "bf16x3": KALDO_BF16X3}

KALDO_DELTA_GAUSS = 0
KALDO_DELTA_LORENTZ = 1
KALDO_DELTA_TRIANGLE = 2
DELTAS = {"gauss": KALDO_DELTA_GAUSS, "lorentz": KALDO_DELTA_LORENTZ, "triangle": KALDO_DELTA_TRIANGLE}
KALDO_QUANTUM = 0
KALDO_CLASSICAL = 1
KALDO_MAX_T = 8
KALDO_TUNE_AUTO = 0
KALDO_TUNE_FIXED = 1
KALDO_TUNE_SHAPE0 = 2

STATUS_NAMES = {0: "KALDO_OK", -1: "KALDO_EINVAL", -2: "KALDO_ENOMEM", -3: "KALDO_EDEVICE",
                -4: "KALDO_ESTATE", -5: "KALDO_EUNSTABLE", -6: "KALDO_ENOCONV"}

EXPORTED = ["kaldo_create", "kaldo_destroy", "kaldo_last_error", "kaldo_phonons",
            "kaldo_linewidths", "kaldo_kappa_rta", "kaldo_kappa_qhgk", "kaldo_batch_add",
            "kaldo_batch_run", "kaldo_batch_clear", "kaldo_set_tuning", "kaldo_profile_enable",
            "kaldo_profile_read", "kaldo_phase_space", "kaldo_set_k_range", "kaldo_batch_set_k_range",
            "kaldo_set_workspace", "kaldo_profile_flops", "kaldo_mode_diffusivity",
            "kaldo_kappa_rta_noalloc", "kaldo_kappa_bte", "kaldo_batch_plan", "kaldo_qhgk_options",
            "kaldo_set_gamma", "kaldo_gamma_interpolate", "kaldo_adaptive_width"]


class kaldo_structure(C.Structure):
    _fields_ = [("cell", C.c_double * 9), ("n_atoms", C.c_int32),
                ("positions", C.POINTER(C.c_double)), ("masses", C.POINTER(C.c_double))]


class kaldo_fc2(C.Structure):
    _fields_ = [("n_blocks", C.c_int64), ("i", C.POINTER(C.c_int32)), ("j", C.POINTER(C.c_int32)),
                ("R", C.POINTER(C.c_int32)), ("blocks", C.POINTER(C.c_double))]


class kaldo_fc3(C.Structure):
    _fields_ = [("n_blocks", C.c_int64), ("i", C.POINTER(C.c_int32)), ("j", C.POINTER(C.c_int32)),
                ("l", C.POINTER(C.c_int32)), ("R1", C.POINTER(C.c_int32)), ("R2", C.POINTER(C.c_int32)),
                ("blocks", C.POINTER(C.c_double))]


class KaldoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkaldo.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2009_01967_amd.build`")
    lib = C.CDLL(path)
    lib.kaldo_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]
    lib.kaldo_create.restype = C.c_int
    lib.kaldo_destroy.argtypes = [C.c_void_p]
    lib.kaldo_destroy.restype = None
    lib.kaldo_last_error.argtypes = [C.c_void_p]
    lib.kaldo_last_error.restype = C.c_char_p
    lib.kaldo_phonons.argtypes = [C.c_void_p, C.POINTER(kaldo_structure), C.POINTER(kaldo_fc2),
                                  C.POINTER(C.c_int32), C.c_void_p, C.c_void_p]
    lib.kaldo_phonons.restype = C.c_int
    lib.kaldo_linewidths.argtypes = [C.c_void_p, C.POINTER(kaldo_fc3), C.POINTER(C.c_double), C.c_int32,
                                     C.c_double, C.c_int, C.c_int, C.c_int, C.c_void_p]
    lib.kaldo_linewidths.restype = C.c_int
    lib.kaldo_set_workspace.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.kaldo_set_workspace.restype = C.c_int
    lib.kaldo_set_k_range.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.kaldo_set_k_range.restype = C.c_int
    lib.kaldo_batch_set_k_range.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    lib.kaldo_batch_set_k_range.restype = C.c_int
    lib.kaldo_phase_space.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_int,
                                      C.c_int, C.c_void_p]
    lib.kaldo_phase_space.restype = C.c_int
    lib.kaldo_kappa_rta.argtypes = [C.c_void_p, C.c_void_p]
    lib.kaldo_kappa_rta.restype = C.c_int
    lib.kaldo_kappa_rta_noalloc.argtypes = [C.c_void_p, C.c_void_p]
    lib.kaldo_kappa_rta_noalloc.restype = C.c_int
    lib.kaldo_kappa_bte.argtypes = [C.c_void_p, C.c_int, C.c_int32, C.c_double, C.c_void_p,
                                    C.POINTER(C.c_int32)]
    lib.kaldo_kappa_bte.restype = C.c_int
    lib.kaldo_kappa_qhgk.argtypes = [C.c_void_p, C.c_void_p]
    lib.kaldo_kappa_qhgk.restype = C.c_int
    lib.kaldo_mode_diffusivity.argtypes = [C.c_void_p, C.c_void_p]
    lib.kaldo_mode_diffusivity.restype = C.c_int
    lib.kaldo_adaptive_width.argtypes = [C.c_void_p, C.c_double]
    lib.kaldo_adaptive_width.restype = C.c_int
    lib.kaldo_qhgk_options.argtypes = [C.c_void_p, C.c_double, C.c_double]
    lib.kaldo_qhgk_options.restype = C.c_int
    lib.kaldo_set_gamma.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int, C.c_void_p]
    lib.kaldo_set_gamma.restype = C.c_int
    lib.kaldo_gamma_interpolate.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int, C.c_void_p,
                                            C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    lib.kaldo_gamma_interpolate.restype = C.c_int
    lib.kaldo_batch_add.argtypes = [C.c_void_p, C.POINTER(kaldo_structure), C.POINTER(kaldo_fc2),
                                    C.POINTER(kaldo_fc3), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.kaldo_batch_add.restype = C.c_int
    lib.kaldo_batch_run.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_int, C.c_int,
                                    C.POINTER(C.c_void_p)]
    lib.kaldo_batch_run.restype = C.c_int
    lib.kaldo_batch_plan.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_int, C.c_int]
    lib.kaldo_batch_plan.restype = C.c_int
    lib.kaldo_batch_clear.argtypes = [C.c_void_p]
    lib.kaldo_batch_clear.restype = C.c_int
    lib.kaldo_set_tuning.argtypes = [C.c_void_p, C.c_int]
    lib.kaldo_set_tuning.restype = C.c_int
    lib.kaldo_profile_enable.argtypes = [C.c_void_p, C.c_int]
    lib.kaldo_profile_enable.restype = C.c_int
    lib.kaldo_profile_read.argtypes = [C.c_void_p, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.kaldo_profile_read.restype = C.c_int
    lib.kaldo_profile_flops.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.kaldo_profile_flops.restype = C.c_int
    _lib = lib
    return lib


# ---- same-name thin wrappers ---------------------------------------------------

def kaldo_create(device: int = 0, stream: Optional[int] = None):
    lib = load_library()
    h = C.c_void_p()
    st = lib.kaldo_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
    if st != KALDO_OK:
        raise KaldoError(st, "kaldo_create failed")
    return h


def kaldo_destroy(ctx) -> None:
    load_library().kaldo_destroy(ctx)


def kaldo_last_error(ctx) -> str:
    return load_library().kaldo_last_error(ctx).decode()


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _out_ptr(out):
    """Host numpy array or device tensor (anything with data_ptr) -> void*."""
    if out is None:
        return None
    if hasattr(out, "data_ptr"):
        return C.c_void_p(out.data_ptr())
    return C.c_void_p(out.ctypes.data)


def _check(ctx, st):
    if st != KALDO_OK:
        raise KaldoError(st, kaldo_last_error(ctx))


class _Keep:
    """Holds contiguous copies so ctypes pointers stay valid during a call."""

    def __init__(self):
        self.items = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(a)
        return a


def make_structure(cell, positions, masses, keep: _Keep):
    s = kaldo_structure()
    cell = keep.arr(cell, np.float64).reshape(9)
    for c in range(9):
        s.cell[c] = float(cell[c])
    pos = keep.arr(positions, np.float64)
    m = keep.arr(masses, np.float64)
    s.n_atoms = int(m.shape[0])
    s.positions = _ptr(pos, C.c_double)
    s.masses = _ptr(m, C.c_double)
    return s


def make_fc2(i, j, R, blocks, keep: _Keep):
    f = kaldo_fc2()
    i = keep.arr(i, np.int32)
    f.n_blocks = int(i.shape[0])
    f.i = _ptr(i, C.c_int32)
    f.j = _ptr(keep.arr(j, np.int32), C.c_int32)
    f.R = _ptr(keep.arr(R, np.int32), C.c_int32)
    f.blocks = _ptr(keep.arr(blocks, np.float64), C.c_double)
    return f


def make_fc3(i, j, l, R1, R2, blocks, keep: _Keep):
    f = kaldo_fc3()
    i = keep.arr(i, np.int32)
    f.n_blocks = int(i.shape[0])
    f.i = _ptr(i, C.c_int32)
    f.j = _ptr(keep.arr(j, np.int32), C.c_int32)
    f.l = _ptr(keep.arr(l, np.int32), C.c_int32)
    f.R1 = _ptr(keep.arr(R1, np.int32), C.c_int32)
    f.R2 = _ptr(keep.arr(R2, np.int32), C.c_int32)
    f.blocks = _ptr(keep.arr(blocks, np.float64), C.c_double)
    return f


def kaldo_phonons(ctx, structure, fc2, grid, nu_out=None, vel_out=None) -> int:
    g = (C.c_int32 * 3)(*[int(x) for x in grid])
    return load_library().kaldo_phonons(ctx, C.byref(structure) if structure is not None else None,
                                        C.byref(fc2) if fc2 is not None else None, g,
                                        _out_ptr(nu_out), _out_ptr(vel_out))


def kaldo_linewidths(ctx, fc3, T: Sequence[float], sigma_thz: float, stats: int = KALDO_QUANTUM,
                     precision: int = KALDO_FP64, gamma_out=None, delta: int = KALDO_DELTA_GAUSS) -> int:
    Ts = (C.c_double * max(1, len(T)))(*[float(x) for x in T])
    return load_library().kaldo_linewidths(ctx, C.byref(fc3) if fc3 is not None else None, Ts, len(T),
                                           float(sigma_thz), int(delta), int(stats), int(precision),
                                           _out_ptr(gamma_out))


def kaldo_set_workspace(ctx, dev_ptr: Optional[int], nbytes: int) -> int:
    return load_library().kaldo_set_workspace(ctx, C.c_void_p(dev_ptr) if dev_ptr else None, int(nbytes))


def kaldo_set_k_range(ctx, k_begin: int, k_end: int) -> int:
    return load_library().kaldo_set_k_range(ctx, int(k_begin), int(k_end))


def kaldo_batch_set_k_range(ctx, handle: int, k_begin: int, k_end: int) -> int:
    return load_library().kaldo_batch_set_k_range(ctx, int(handle), int(k_begin), int(k_end))


def kaldo_phase_space(ctx, T: Sequence[float], sigma_thz: float, delta: int = KALDO_DELTA_GAUSS,
                      stats: int = KALDO_QUANTUM, g_out=None) -> int:
    Ts = (C.c_double * max(1, len(T)))(*[float(x) for x in T])
    return load_library().kaldo_phase_space(ctx, Ts, len(T), float(sigma_thz), int(delta), int(stats),
                                            _out_ptr(g_out))


def kaldo_kappa_rta(ctx, kappa_out=None) -> int:
    return load_library().kaldo_kappa_rta(ctx, _out_ptr(kappa_out))


def kaldo_kappa_rta_noalloc(ctx, kappa_out) -> int:
    return load_library().kaldo_kappa_rta_noalloc(ctx, _out_ptr(kappa_out))


def kaldo_kappa_bte(ctx, method: int, max_terms: int, tol: float, kappa_out, terms_out=None) -> int:
    """terms_out: a one-element int32 numpy array, or None."""
    tp = None if terms_out is None else terms_out.ctypes.data_as(C.POINTER(C.c_int32))
    return load_library().kaldo_kappa_bte(ctx, int(method), int(max_terms), float(tol), _out_ptr(kappa_out), tp)


def kaldo_kappa_qhgk(ctx, kappa_out=None) -> int:
    return load_library().kaldo_kappa_qhgk(ctx, _out_ptr(kappa_out))


def kaldo_mode_diffusivity(ctx, d_out) -> int:
    return load_library().kaldo_mode_diffusivity(ctx, _out_ptr(d_out))


def kaldo_adaptive_width(ctx, scale: float) -> int:
    return load_library().kaldo_adaptive_width(ctx, float(scale))


def kaldo_qhgk_options(ctx, bandwidth: float = 0.0, threshold: float = 0.0) -> int:
    return load_library().kaldo_qhgk_options(ctx, float(bandwidth), float(threshold))


def _in_ptr(a, keep):
    """Host array (made contiguous float64 and kept alive) or device tensor -> void*."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(keep.arr(a, np.float64).ctypes.data)


def kaldo_set_gamma(ctx, T: Sequence[float], stats: int, gamma) -> int:
    keep = _Keep()
    Ts = (C.c_double * max(1, len(T)))(*[float(x) for x in T])
    return load_library().kaldo_set_gamma(ctx, Ts, len(T), int(stats), _in_ptr(gamma, keep))


def kaldo_gamma_interpolate(ctx, T: Sequence[float], stats: int, omega_src, gamma_src, n_src: int,
                            n_bins: int, gamma_out=None) -> int:
    keep = _Keep()
    Ts = (C.c_double * max(1, len(T)))(*[float(x) for x in T])
    return load_library().kaldo_gamma_interpolate(ctx, Ts, len(T), int(stats), _in_ptr(omega_src, keep),
                                                  _in_ptr(gamma_src, keep), int(n_src), int(n_bins),
                                                  _out_ptr(gamma_out))


def kaldo_batch_add(ctx, structure, fc2, fc3, grid):
    """Add one crystal to the context's batch; returns (status, handle)."""
    g = (C.c_int32 * 3)(*[int(x) for x in grid])
    h = C.c_int32(-1)
    st = load_library().kaldo_batch_add(ctx, C.byref(structure), C.byref(fc2), C.byref(fc3), g, C.byref(h))
    return st, h.value


def kaldo_batch_run(ctx, T: Sequence[float], sigma_thz: float, stats: int, precision: int, gamma_outs) -> int:
    """gamma_outs: one output (numpy array, device tensor or None) per crystal, or None."""
    Ts = (C.c_double * max(1, len(T)))(*[float(x) for x in T])
    arr = None
    if gamma_outs is not None:
        arr = (C.c_void_p * max(1, len(gamma_outs)))()
        for i, o in enumerate(gamma_outs):
            p = _out_ptr(o)
            arr[i] = p.value if p is not None else None
    return load_library().kaldo_batch_run(ctx, Ts, len(T), float(sigma_thz), int(stats), int(precision), arr)


def kaldo_batch_plan(ctx, T: Sequence[float], sigma_thz: float, stats: int, precision: int) -> int:
    Ts = (C.c_double * max(1, len(T)))(*[float(x) for x in T])
    return load_library().kaldo_batch_plan(ctx, Ts, len(T), float(sigma_thz), int(stats), int(precision))


def kaldo_batch_clear(ctx) -> int:
    return load_library().kaldo_batch_clear(ctx)


def kaldo_set_tuning(ctx, mode: int) -> int:
    """KALDO_TUNE_AUTO (0), KALDO_TUNE_FIXED (1) or KALDO_TUNE_SHAPE0 + v (tile shape v)."""
    return load_library().kaldo_set_tuning(ctx, int(mode))


def kaldo_profile_enable(ctx, enable: bool = True) -> int:
    return load_library().kaldo_profile_enable(ctx, 1 if enable else 0)


def kaldo_profile_read(ctx, kernel: str):
    """(total_ms, launches) of a named kernel since profiling was enabled."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    st = load_library().kaldo_profile_read(ctx, kernel.encode(), C.byref(ms), C.byref(n))
    _check(ctx, st)
    return ms.value, n.value


def kaldo_profile_flops(ctx):
    """(executed, dense) projection-GEMM matrix-core flops since profiling was enabled."""
    ex = C.c_double(0.0)
    dn = C.c_double(0.0)
    _check(ctx, load_library().kaldo_profile_flops(ctx, C.byref(ex), C.byref(dn)))
    return ex.value, dn.value


# ---- convenience context ---------------------------------------------------------

class Context:
    """One library context on one GPU.  Inputs are numpy arrays; outputs are
    numpy arrays unless a device tensor is passed as ``out``."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, workspace=None):
        """``workspace``: device memory for every buffer of the context
        (kaldo_set_workspace): a CUDA uint8 torch tensor, kept alive by the
        context, or a (device pointer, bytes) pair.  As with torch streams,
        torch must have initialised the GPU before the library's first call in
        the process (the library and torch each load a HIP runtime)."""
        self.h = kaldo_create(device, stream)
        self.nk = 0
        self.n = 0
        self.nT = 0
        self.workspace = workspace
        if workspace is not None:
            if isinstance(workspace, tuple):
                ptr, nbytes = workspace
            else:
                ptr, nbytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
            _check(self.h, kaldo_set_workspace(self.h, ptr, nbytes))

    def close(self):
        if self.h:
            kaldo_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def phonons(self, crystal=None, grid=None, nu_out=None, vel_out=None, want_host=True):
        """Upload structure + fc2 of ``crystal`` (or reuse the resident ones when
        crystal is None) and compute the modes on ``grid``."""
        keep = _Keep()
        s = f2 = None
        if crystal is not None:
            s = make_structure(crystal.cell, crystal.positions, crystal.masses, keep)
            f2 = make_fc2(crystal.fc2_i, crystal.fc2_j, crystal.fc2_R, crystal.fc2_val, keep)
            self.n = 3 * crystal.n_atoms
            grid = crystal.grid if grid is None else grid
        grid = tuple(int(x) for x in grid)
        self.nk = int(np.prod(grid))
        if want_host and nu_out is None:
            nu_out = np.zeros((self.nk, self.n))
        _check(self.h, kaldo_phonons(self.h, s, f2, grid, nu_out, vel_out))
        return nu_out

    def linewidths(self, crystal=None, T=(300.0,), sigma_thz=0.1, precision="fp64", classical=False,
                   gamma_out=None, want_host=True, delta="gauss"):
        keep = _Keep()
        f3 = None
        if crystal is not None:
            f3 = make_fc3(crystal.fc3_i, crystal.fc3_j, crystal.fc3_l, crystal.fc3_R1, crystal.fc3_R2,
                          crystal.fc3_val, keep)
        self.nT = len(T)
        if want_host and gamma_out is None:
            gamma_out = np.zeros((len(T), self.nk, self.n))
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(self.h, kaldo_linewidths(self.h, f3, T, sigma_thz,
                                        KALDO_CLASSICAL if classical else KALDO_QUANTUM, prec, gamma_out,
                                        delta=DELTAS[delta] if isinstance(delta, str) else int(delta)))
        return gamma_out

    def batch_add(self, crystal) -> int:
        """Add a crystal (its modes are computed now, on crystal.grid); returns its handle."""
        keep = _Keep()
        s = make_structure(crystal.cell, crystal.positions, crystal.masses, keep)
        f2 = make_fc2(crystal.fc2_i, crystal.fc2_j, crystal.fc2_R, crystal.fc2_val, keep)
        f3 = make_fc3(crystal.fc3_i, crystal.fc3_j, crystal.fc3_l, crystal.fc3_R1, crystal.fc3_R2,
                      crystal.fc3_val, keep)
        st, h = kaldo_batch_add(self.h, s, f2, f3, crystal.grid)
        _check(self.h, st)
        if not hasattr(self, "batch_shapes"):
            self.batch_shapes = []
        self.batch_shapes.append((int(np.prod(crystal.grid)), 3 * crystal.n_atoms))
        return h

    def batch_run(self, T=(300.0,), sigma_thz=0.1, precision="fp32", classical=False, outs=None):
        """Linewidths of every crystal of the batch (one graph launch); returns
        the list of per-crystal outputs ([nT][Nk][n] numpy arrays by default)."""
        if outs is None:
            outs = [np.zeros((len(T), nk, n)) for nk, n in getattr(self, "batch_shapes", [])]
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(self.h, kaldo_batch_run(self.h, T, sigma_thz, KALDO_CLASSICAL if classical else KALDO_QUANTUM,
                                       prec, outs))
        return outs

    def batch_clear(self):
        _check(self.h, kaldo_batch_clear(self.h))
        self.batch_shapes = []

    def set_k_range(self, k_begin=0, k_end=2**31 - 1):
        """Compute later linewidths for first-mode points k_begin <= k < k_end only."""
        _check(self.h, kaldo_set_k_range(self.h, k_begin, k_end))

    def batch_set_k_range(self, handle, k_begin, k_end):
        _check(self.h, kaldo_batch_set_k_range(self.h, handle, k_begin, k_end))

    def phase_space(self, T=(300.0,), sigma_thz=0.1, classical=False, delta="gauss", out=None):
        """Phase space per mode g [nT][Nk][n] in ps/rad on the last phonons' grid."""
        if out is None:
            out = np.zeros((len(T), self.nk, self.n))
        _check(self.h, kaldo_phase_space(self.h, T, sigma_thz,
                                         DELTAS[delta] if isinstance(delta, str) else int(delta),
                                         KALDO_CLASSICAL if classical else KALDO_QUANTUM, out))
        return out

    def kappa_bte(self, method="inverse", max_terms=500, tol=1e-14):
        """Full linearised BTE conductivity [nT][3][3] W/(m K) for the last
        linewidths: returns (kappa, terms, converged).  A series that has not
        converged returns its last partial sum with converged False."""
        out = np.zeros((self.nT, 3, 3))
        terms = np.zeros(1, dtype=np.int32)
        st = kaldo_kappa_bte(self.h, BTE_METHODS[method] if isinstance(method, str) else int(method),
                             max_terms, tol, out, terms)
        if st not in (KALDO_OK, KALDO_ENOCONV):
            _check(self.h, st)
        return out, int(terms[0]), st == KALDO_OK

    def kappa_rta(self, out=None, want_host=True):
        if want_host and out is None:
            out = np.zeros((self.nT, 3, 3))
        _check(self.h, kaldo_kappa_rta(self.h, out))
        return out

    def kappa_qhgk(self, out=None, want_host=True):
        if want_host and out is None:
            out = np.zeros((self.nT, 3, 3))
        _check(self.h, kaldo_kappa_qhgk(self.h, out))
        return out

    def adaptive_width(self, scale=1.0):
        """Per-process Gaussian widths from the velocities for later linewidths
        (scale 0 turns them off); the linewidths' sigma_thz is the smallest width."""
        _check(self.h, kaldo_adaptive_width(self.h, scale))

    def qhgk_options(self, bandwidth=0.0, threshold=0.0):
        """QHGK bandwidth eta and energy threshold [rad/ps] for later kappa_qhgk
        and mode_diffusivity calls (0 turns each off)."""
        _check(self.h, kaldo_qhgk_options(self.h, bandwidth, threshold))

    def set_gamma(self, T=(300.0,), gamma=None, classical=False):
        """Install linewidths [nT][Nk][n] (host array or device tensor; None: zeros)."""
        _check(self.h, kaldo_set_gamma(self.h, T, KALDO_CLASSICAL if classical else KALDO_QUANTUM, gamma))
        self.nT = len(T)

    def gamma_interpolate(self, omega_src, gamma_src, n_bins=64, T=(300.0,), classical=False, gamma_out=None,
                          want_host=True):
        """Linewidths of this context's modes from gamma(omega) of source modes:
        omega_src [n_src] rad/ps, gamma_src [nT][n_src] rad/ps (host arrays or
        device tensors).  Returns the interpolated [nT][Nk][n] linewidths."""
        n_src = int(omega_src.shape[0]) if hasattr(omega_src, "shape") else len(omega_src)
        if want_host and gamma_out is None:
            gamma_out = np.zeros((len(T), self.nk, self.n))
        _check(self.h, kaldo_gamma_interpolate(self.h, T, KALDO_CLASSICAL if classical else KALDO_QUANTUM,
                                               omega_src, gamma_src, n_src, n_bins, gamma_out))
        self.nT = len(T)
        return gamma_out

    def mode_diffusivity(self, out=None):
        """[nT][n][3] mode diffusivity at Gamma in mm^2/s (host array unless a
        device tensor is given)."""
        if out is None:
            out = np.zeros((self.nT, self.n, 3))
        _check(self.h, kaldo_mode_diffusivity(self.h, out))
        return out
