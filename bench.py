"""Benchmark of the three-phonon linewidth path on one MI355X.

Headline (one step): the linewidths of every mode of the 32-crystal batch
(cells of 2..54 atoms, grids 4^3..10^3, Si/Ge masses, T = 300 K, Gaussian
delta of 0.1 THz) in FP32, as one launch of the batch's HIP graph: a single
persistent kernel works through the cost-sorted table of (crystal, first-mode
point, partner range) rounds of every many-branch crystal.  Inputs are resident
(harmonic modes computed and the graph planned and captured before timing).
FP64 is timed beside it on a share of each crystal's first-mode points.

Sections beside the headline: the 2-atom diamond cell on 16^3 (the few-branch
VALU kernel, FP32 and FP64 steps with phonons and RTA conductivity), the
many-branch workloads (46-atom cage cell on 5x5x5 and the 1000-atom SiGe cell
at Gamma; BF16X3, FP32 and FP64 in a child process), the full linearised BTE
and the delta/phase-space variants on the diamond cell, the attainable unit
peaks and the CPU oracle on a sample of the batch.

Prints one JSON line.  ``--gpus`` above 1 is refused: one GPU only.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "diamond-2at-16x16x16-shell3"
BATCH_WORKLOAD = "batch-32-crystals-2..54at-4^3..10^3"
METRIC = "phonon linewidths/s + projection TFLOP/s, mixed vs FP64, at rel err ≤1e-4"
FP32_VECTOR_PEAK = 157.3e12     # MI355X published vector FP32 (FLOP/s)
FP64_VECTOR_PEAK = 78.6e12
BF16_MFMA_PEAK = 2.5e15         # dense bf16 MFMA
FP32_MFMA_PEAK = 157.3e12
FP64_MFMA_PEAK = 78.6e12
MFMA_WORKLOADS = ("cage-46at-5x5x5", "sige-1000at-gamma")
# HBM bytes per launch of the headline kernel (k_batch_persistent<1,1>, the
# full draw): rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE over this benchmark
# (--no-cpu --no-mfma --no-c2), each scaled by what the counter reads for a
# plain 1 GiB device copy (--copy-calibration: FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0).  Set to None when that kernel changes.
HEADLINE_TRAFFIC = {"fetch_bytes": 144395413575 * 1024 * 2.0, "write_bytes": 85815321664 * 1024 * 1.0}
# The same for the few-branch kernel k_project_small<float,6,3,true,0> on the
# 2-atom diamond cell (--c2-only, KiB per dispatch, same scales).
C2_TRAFFIC = {"fetch_bytes": 53591.0 * 1024 * 2.0, "write_bytes": 5115.8 * 1024 * 1.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def computed_points(grid):
    """First-mode points a whole-grid linewidth pass computes: one of each pair
    (k, -k) (the linewidth is even under time reversal; the library copies the
    values to the other point), i.e. (N_k + number of points with k = -k) / 2."""
    g = [int(x) for x in grid]
    self_mirror = 1
    for x in g:
        self_mirror *= 2 if x % 2 == 0 else 1
    return (int(np.prod(g)) + self_mirror) // 2


def shared_points(grid, m):
    """First-mode points computed for the range [0, m) of a grid: the distinct
    representatives min(k, -k) of its points."""
    g = [int(x) for x in grid]
    reps = set()
    for k in range(m):
        m0, m1, m2 = k // (g[1] * g[2]), (k // g[2]) % g[1], k % g[2]
        km = (((-m0) % g[0]) * g[1] + (-m1) % g[1]) * g[2] + (-m2) % g[2]
        reps.add(min(k, km))
    return len(reps)


def algorithmic_flops(nk, n, nd, npts=None):
    """Projection work of one linewidth pass over npts first-mode points (steps
    B and C, one V for both signs): per point 8 N_k N_Delta n^3 + 16 N_k n^4."""
    npts = nk if npts is None else npts
    f_b = 8.0 * npts * nk * nd * n ** 3
    f_c = 16.0 * npts * nk * n ** 4
    return f_b, f_c


def intermediate_bytes(nk, n, nd, nT, npts):
    """Bytes the projection kernel reads and writes once (FP32 path): its step-A
    intermediate, eigenvectors, Delta phases, mode tables and the partial sums
    (the implementation's traffic, not the method's unique inputs)."""
    a = npts * n * nd * n * n * 8        # A_k[s][Delta][a'][a''] complex float
    et = n * n * nk * 8                  # eigenvectors, complex float
    ph = nd * nk * 8                     # phases, complex float
    tab = (2 + nT) * n * nk * 8          # omega, 1/omega, occupations (double)
    part = npts * (nk // 256) * nT * n * 8  # per-tile partial sums (double)
    return float(a + et + ph + tab + part)


def survey_algorithmic_bytes(c, nT):
    """The method's unique inputs and outputs: eigenvectors (complex double),
    fc3 blocks and the linewidths."""
    return float(c.n_k * c.n_modes ** 2 * 16 + len(c.fc3_i) * 27 * 8 + nT * c.n_k * c.n_modes * 8)


def run_c2(steps=20, warmup=3):
    """The 2-atom diamond cell on 16^3 (few-branch VALU kernel): FP32 and FP64
    steps of phonons + linewidths + RTA conductivity on resident inputs."""
    import torch
    from gen import workload, WORKLOADS
    from paper_2009_01967_amd import kaldo

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    w = WORKLOADS[WORKLOAD]
    c = workload(WORKLOAD)
    T = list(w["T"])
    sigma = w["sigma_thz"]
    nk, n = c.n_k, c.n_modes
    dev = torch.device("cuda:0")
    # a torch-owned stream (default priority); the library launches on it and
    # the timing events are recorded on it
    stream = torch.cuda.Stream(device=dev)
    ctx = kaldo.Context(0, stream.cuda_stream)
    # upload the inputs once; later calls pass NULL and reuse the resident copies
    ctx.phonons(c)
    ctx.linewidths(c, T=T, sigma_thz=sigma, precision="fp64")
    nu_d = torch.empty((nk, n), dtype=torch.float64, device=dev)
    g_d = torch.empty((len(T), nk, n), dtype=torch.float64, device=dev)
    k_d = torch.empty((len(T), 3, 3), dtype=torch.float64, device=dev)

    def step(prec):
        h = ctx.h
        kaldo._check(h, kaldo.kaldo_phonons(h, None, None, c.grid, nu_d, None))
        kaldo._check(h, kaldo.kaldo_linewidths(h, None, T, sigma, kaldo.KALDO_QUANTUM, prec, g_d))
        kaldo._check(h, kaldo.kaldo_kappa_rta(h, k_d))

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        kaldo.kaldo_profile_enable(ctx.h, True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step(prec)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        ms = e0.elapsed_time(e1) / steps
        kern = {}
        for name in ("dyn_assemble", "eigensolve", "step_a", "project", "finalize", "kappa_rta"):
            tot, cnt = kaldo.kaldo_profile_read(ctx.h, name)
            kern[name] = {"avg_ms": tot / cnt if cnt else None, "launches": cnt}
        kaldo.kaldo_profile_enable(ctx.h, False)
        return ms, wall, kern, g_d.cpu().numpy().copy(), k_d.cpu().numpy().copy()

    ms32, wall32, kern32, g32, k32 = timed(kaldo.KALDO_FP32, steps, warmup)
    log(f"fp32: {ms32:.3f} ms/step (wall {wall32:.3f}), kernels {kern32}")
    ms64, wall64, kern64, g64, k64 = timed(kaldo.KALDO_FP64, max(2, steps // 2), 1)
    log(f"fp64: {ms64:.3f} ms/step (wall {wall64:.3f}), kernels {kern64}")
    dset = {tuple(int(v) for v in x) for x in (c.fc3_R2 - c.fc3_R1)}
    nd = len(dset)
    # (Delta, -Delta) pairs, Delta != 0: the FP32 step B sums each with two real multiplies
    npair = sum(1 for x in dset if x > (0, 0, 0) and tuple(-v for v in x) in dset)
    ctx.close()
    return dict(c=c, w=w, T=T, sigma=sigma, nk=nk, n=n, nd=nd, npair=npair, ms32=ms32, ms64=ms64, wall32=wall32,
                wall64=wall64, kern32=kern32, kern64=kern64, g32=g32, g64=g64, k32=k32, k64=k64)


def qhgk_options_section(ctx, c, T, sigma, stream, steps):
    """The QHGK options of Appendix A on a Gamma cell whose FP64 linewidths are
    resident: kappa_QHGK with every pair, with an energy threshold, with a
    bandwidth (Allen-Feldman), and from linewidths interpolated in frequency
    from the smaller cell of the same alloy (3^3 instead of 5^3 conventional
    cells), whose linewidths the GPU computes here (FP32)."""
    import torch
    from gen import sige_supercell
    from paper_2009_01967_amd import kaldo

    def timed_kappa():
        kaldo.kaldo_profile_enable(ctx.h, True)
        for _ in range(steps):
            k = ctx.kappa_qhgk()
        tot, cnt = kaldo.kaldo_profile_read(ctx.h, "kappa_qhgk")
        kaldo.kaldo_profile_enable(ctx.h, False)
        return k, tot / max(cnt, 1)

    n = c.n_modes
    w = 2.0 * np.pi * ctx.phonons(None, grid=c.grid)[0]
    g64 = np.zeros((len(T), 1, n))
    kaldo._check(ctx.h, kaldo.kaldo_linewidths(ctx.h, None, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP64, g64))
    k_all, ms_all = timed_kappa()
    out = {"kappa_xx_all_pairs": float(k_all[0, 0, 0]), "pair_sum_ms_all": ms_all}
    dw = np.abs(w[:, None] - w[None, :])
    for thr in (1.0, 4.0):
        ctx.qhgk_options(threshold=thr)
        k, ms = timed_kappa()
        out[f"threshold_{thr:g}_rad_ps"] = {"kappa_rel_change": float(np.abs(k - k_all).max() / np.abs(k_all).max()),
                                            "pairs_kept_frac": float(np.mean(dw <= thr)), "pair_sum_ms": ms}
    ctx.qhgk_options()
    eta = 0.5
    ctx.qhgk_options(bandwidth=eta)
    k_af, ms = timed_kappa()
    ctx.qhgk_options()
    out["allen_feldman_bandwidth_0.5_rad_ps"] = {"kappa_xx": float(k_af[0, 0, 0]), "pair_sum_ms": ms}
    # interpolation from the 216-atom cell
    small = sige_supercell(reps=3)
    sctx = kaldo.Context(0, stream.cuda_stream)
    nu_s = sctx.phonons(small)
    sctx.linewidths(small, T=T, sigma_thz=sigma, precision="fp32")   # uploads fc3, tunes the tiles
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_s = sctx.linewidths(None, T=T, sigma_thz=sigma, precision="fp32")
    small_ms = (time.perf_counter() - t0) * 1e3
    sctx.close()
    kaldo.kaldo_profile_enable(ctx.h, True)
    gi = ctx.gamma_interpolate(2.0 * np.pi * nu_s.reshape(-1), g_s.reshape(len(T), -1), n_bins=48, T=T)
    tot, cnt = kaldo.kaldo_profile_read(ctx.h, "gamma_interpolate")
    kaldo.kaldo_profile_enable(ctx.h, False)
    k_i, _ = timed_kappa()
    mask = g64 > 0
    out["interpolated_from_216_atoms"] = {
        "n_bins": 48, "small_cell_linewidths_ms": small_ms, "interpolate_ms": tot / max(cnt, 1),
        "kappa_rel_diff_vs_computed_gamma": float(np.abs(k_i - k_all).max() / np.abs(k_all).max()),
        "gamma_median_rel_diff": float(np.median(np.abs(gi[mask] - g64[mask]) / g64[mask]))}
    # leave the computed FP64 linewidths resident again
    kaldo._check(ctx.h, kaldo.kaldo_linewidths(ctx.h, None, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP64, None))
    log(f"qhgk options: {out}")
    return out


def run_mfma(name, steps, warmup):
    """Linewidths and kappa of a many-branch workload on resident phonons, BF16X3,
    FP32 and FP64, with the projection GEMMs timed through the library's hooks;
    one phonon pass is timed on its own."""
    import torch
    from gen import workload, WORKLOADS
    from paper_2009_01967_amd import kaldo

    w = WORKLOADS[name]
    t0 = time.perf_counter()
    c = workload(name)
    log(f"{name}: generated in {time.perf_counter() - t0:.1f} s")
    T, sigma = list(w["T"]), w["sigma_thz"]
    nk, n = c.n_k, c.n_modes
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ctx = kaldo.Context(0, stream.cuda_stream)
    ctx.phonons(c)
    ctx.linewidths(c, T=T, sigma_thz=sigma, precision="bf16x3")
    g_d = torch.empty((len(T), nk, n), dtype=torch.float64, device=dev)
    k_d = torch.empty((len(T), 3, 3), dtype=torch.float64, device=dev)
    kappa = kaldo.kaldo_kappa_qhgk if nk == 1 else kaldo.kaldo_kappa_rta

    def step(prec):
        h = ctx.h
        kaldo._check(h, kaldo.kaldo_linewidths(h, None, T, sigma, kaldo.KALDO_QUANTUM, prec, g_d))
        kaldo._check(h, kappa(h, k_d))

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    kaldo._check(ctx.h, kaldo.kaldo_phonons(ctx.h, None, None, c.grid, None, None))
    e1.record(stream)
    torch.cuda.synchronize()
    phonon_ms = e0.elapsed_time(e1)
    res = {}
    for label, prec in (("bf16x3", kaldo.KALDO_BF16X3), ("fp32", kaldo.KALDO_FP32), ("fp64", kaldo.KALDO_FP64)):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        kaldo.kaldo_profile_enable(ctx.h, True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step(prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        kern = {}
        for kname in ("eigensolve", "step_a", "step_b", "gamma_sparse", "project"):
            tot, cnt = kaldo.kaldo_profile_read(ctx.h, kname)
            if cnt:
                kern[kname] = {"ms_per_step": tot / steps, "launches_per_step": cnt / steps}
        ex, dense = kaldo.kaldo_profile_flops(ctx.h)
        kaldo.kaldo_profile_enable(ctx.h, False)
        res[label] = dict(ms=ms, kern=kern, ex=ex / steps, dense=dense / steps,
                          g=g_d.cpu().numpy().copy(), k=k_d.cpu().numpy().copy())
        log(f"{name} {label}: {ms:.2f} ms/step, kernels {kern}")
    diff = None
    if nk == 1:
        # mode diffusivity from the FP64 linewidths of the last step: one call
        # is the velocity matrices (three pairs of n x n FP64 GEMMs) plus the
        # pair sum; the pair sum reads V_d (3 n^2 doubles) once per temperature
        d_d = torch.empty((len(T), n, 3), dtype=torch.float64, device=dev)
        kaldo._check(ctx.h, kaldo.kaldo_mode_diffusivity(ctx.h, d_d))
        torch.cuda.synchronize()
        kaldo.kaldo_profile_enable(ctx.h, True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            kaldo._check(ctx.h, kaldo.kaldo_mode_diffusivity(ctx.h, d_d))
        e1.record(stream)
        torch.cuda.synchronize()
        tot, cnt = kaldo.kaldo_profile_read(ctx.h, "diffusivity")
        kaldo.kaldo_profile_enable(ctx.h, False)
        kms = tot / max(cnt, 1)
        nbytes = len(T) * 3.0 * n * n * 8 + len(T) * n * 3 * 8
        diff = {"ms_per_call": e0.elapsed_time(e1) / steps, "pair_sum_ms": kms,
                "roofline": {"bound": "hbm", "kernel": "k_qhgk_diffusivity + k_diffusivity_reduce",
                             "achieved": nbytes / (kms * 1e-3) / 1e9 if kms else None, "peak": 8000.0,
                             "unit": "GB/s", "frac": nbytes / (kms * 1e-3) / 8e12 if kms else None,
                             "traffic": None, "bytes_per_launch": nbytes}}
        log(f"{name} mode diffusivity: {diff['ms_per_call']:.3f} ms per call, pair sum {kms:.3f} ms")
        diff["qhgk_options"] = qhgk_options_section(ctx, c, T, sigma, stream, steps)
    ctx.close()
    lw = nk * n * len(T)
    # algorithmic GEMM flops of the computed first-mode points, one V for both signs
    f_c = 16.0 * computed_points(c.grid) * nk * n ** 4 if nk > 1 else 2.0 * n ** 4
    g64 = res["fp64"]["g"]
    floor = 1e-6 * np.abs(g64).max()
    err = float(np.max(np.abs(res["bf16x3"]["g"] - g64) / np.maximum(np.abs(g64), floor)))
    kerr = float(np.max(np.abs(res["bf16x3"]["k"] - res["fp64"]["k"])) / np.abs(res["fp64"]["k"]).max())
    err32 = float(np.max(np.abs(res["fp32"]["g"] - g64) / np.maximum(np.abs(g64), floor)))
    out = {"workload": name, "n_k": nk, "n_modes": n, "T_K": T, "sigma_thz": sigma,
           "step": "kaldo_linewidths + kaldo_kappa on resident phonons", "phonons_ms": phonon_ms,
           "gemm_flops_per_step": f_c, "gamma_rel_err_bf16x3_vs_fp64": err,
           "kappa_rel_err_bf16x3_vs_fp64": kerr, "gamma_rel_err_fp32_vs_fp64": err32}
    for label, peak in (("bf16x3", BF16_MFMA_PEAK), ("fp32", FP32_MFMA_PEAK), ("fp64", FP64_MFMA_PEAK)):
        ms = res[label]["ms"]
        proj = res[label]["kern"].get("project", {}).get("ms_per_step")
        ent = {"ms_per_step": ms, "value": lw / (ms * 1e-3), "unit": "linewidths/s",
               "kernels_ms_per_step": {k: v["ms_per_step"] for k, v in res[label]["kern"].items()}}
        if proj:
            # The library's tally gives the matrix-core flops of the block tiles
            # that ran and of all tiles launched (tiles whose outputs all lie
            # beyond the delta cut are skipped); both include the padding of the
            # tiles.  achieved = algorithmic F_C x (fraction of the tiled work
            # that ran) / time: the useful rate, padding and screened tiles
            # excluded.  BF16X3 issues three bf16 products per FP32-accurate
            # product, so its peak is a third of the bf16 one; the issued rate
            # is also given against the instruction's own dense peak.
            mult = 3.0 if label == "bf16x3" else 1.0
            ex, dense = res[label]["ex"], res[label]["dense"]
            sec = proj * 1e-3
            ran = ex / dense if dense else 1.0
            ent["roofline"] = {"bound": "mfma", "kernel": "k_gemm (projection GEMMs, fused epilogue)",
                               "achieved": f_c * ran / sec / 1e12, "peak": peak / mult / 1e12, "unit": "TFLOP/s",
                               "frac": f_c * ran / sec / (peak / mult), "traffic": None,
                               "basis": "algorithmic GEMM flops of the tiles that ran (library tally)",
                               "tiles_skipped_frac": 1.0 - ran,
                               "mfma_tflops_issued": ex / sec / 1e12, "mfma_issued_frac": ex / sec / peak,
                               "dense_equivalent_tflops": f_c / sec / 1e12}
        out[label] = ent
    if diff is not None:
        out["mode_diffusivity"] = diff
    out["speedup_bf16x3_vs_fp64"] = res["fp64"]["ms"] / res["bf16x3"]["ms"]
    out["speedup_fp32_vs_fp64"] = res["fp64"]["ms"] / res["fp32"]["ms"]
    return out


def batch_flops(c, npts):
    """Algorithmic flops (F_A, F_B, F_C) of npts first-mode points of crystal c."""
    n, nk = c.n_modes, c.n_k
    nd = len({tuple(int(v) for v in x) for x in (c.fc3_R2 - c.fc3_R1)})
    nnz = 27 * len(c.fc3_i)
    return 4.0 * npts * n * nnz, 8.0 * npts * nk * nd * n ** 3, 16.0 * npts * nk * n ** 4


def run_batch_headline(steps, warmup, div=64, share=1):
    """The headline: linewidths of every mode of the 32-crystal batch in FP32,
    one graph launch (the persistent kernel) per step (share > 1: only the
    first ceil(N_k / share) first-mode points of each crystal, for a shorter
    run); FP64 beside it on the first ceil(N_k / div) points of each crystal."""
    import torch
    from gen import batch_crystals
    from paper_2009_01967_amd import kaldo

    t0 = time.perf_counter()
    crystals = batch_crystals()
    log(f"batch: {len(crystals)} crystals generated in {time.perf_counter() - t0:.1f} s")
    T, sigma = [300.0], 0.1
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    out = {}
    # ---- FP32, every first-mode point
    ctx = kaldo.Context(0, stream.cuda_stream)
    t0 = time.perf_counter()
    share_pts = [c.n_k if share == 1 else max(1, -(-c.n_k // share)) for c in crystals]
    for i, c in enumerate(crystals):
        ctx.batch_add(c)
        if share != 1:
            ctx.batch_set_k_range(i, 0, share_pts[i])
    torch.cuda.synchronize()
    phonon_s = time.perf_counter() - t0
    log(f"batch fp32: phonons of {len(crystals)} crystals in {phonon_s:.1f} s")
    g32 = [np.zeros((len(T), c.n_k, c.n_modes)) for c in crystals]
    t0 = time.perf_counter()
    kaldo._check(ctx.h, kaldo.kaldo_batch_plan(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP32))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"batch fp32: planned and captured in {setup_s:.1f} s")
    for _ in range(warmup):
        kaldo._check(ctx.h, kaldo.kaldo_batch_run(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP32, None))
    torch.cuda.synchronize()
    kaldo.kaldo_profile_enable(ctx.h, True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        kaldo._check(ctx.h, kaldo.kaldo_batch_run(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP32,
                                                   g32 if i == steps - 1 else None))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) * 1e3 / steps
    ms = e0.elapsed_time(e1) / steps
    graph_ms, launches = kaldo.kaldo_profile_read(ctx.h, "batch_graph")
    phases = {}
    for name in ("batch_a_collect", "batch_step_b", "batch_gemm1", "batch_gemm2", "batch_barrier_wait",
                 "batch_wait_gemm1_phase", "batch_wait_gemm2_phase", "batch_set_average"):
        tot, cnt = kaldo.kaldo_profile_read(ctx.h, name)
        phases[name] = tot / max(cnt, 1)
    log(f"batch fp32 phases (ms per launch, workgroup 0): {phases}")
    per_crystal = {}
    for i in range(len(crystals)):
        tot, cnt = kaldo.kaldo_profile_read(ctx.h, f"batch_crystal_{i}")
        if cnt:
            per_crystal[i] = tot / cnt
    ex, dense = kaldo.kaldo_profile_flops(ctx.h)
    kaldo.kaldo_profile_enable(ctx.h, False)
    ctx.close()
    log(f"batch fp32: {ms:.1f} ms per launch (wall {wall:.1f}), graph {graph_ms / max(launches, 1):.1f} ms, "
        f"tiles run {ex / dense if dense else 1.0:.3f}")
    # ---- FP64 beside it on a share of the points
    sub = [max(1, -(-c.n_k // div)) for c in crystals]
    ctx = kaldo.Context(0, stream.cuda_stream)
    for i, (c, m) in enumerate(zip(crystals, sub)):
        ctx.batch_add(c)
        ctx.batch_set_k_range(i, 0, m)
    g64 = [np.zeros((len(T), c.n_k, c.n_modes)) for c in crystals]
    kaldo._check(ctx.h, kaldo.kaldo_batch_run(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP64, g64))
    torch.cuda.synchronize()
    f0 = torch.cuda.Event(enable_timing=True)
    f1 = torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    kaldo._check(ctx.h, kaldo.kaldo_batch_run(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP64, None))
    f1.record(stream)
    torch.cuda.synchronize()
    ms64 = f0.elapsed_time(f1)
    ctx.close()
    log(f"batch fp64 (first ceil(N_k/{div}) points): {ms64:.1f} ms per launch")
    # ---- BF16X3 on the same points
    ctx = kaldo.Context(0, stream.cuda_stream)
    for i, (c, m) in enumerate(zip(crystals, sub)):
        ctx.batch_add(c)
        ctx.batch_set_k_range(i, 0, m)
    gbf = [np.zeros((len(T), c.n_k, c.n_modes)) for c in crystals]
    kaldo._check(ctx.h, kaldo.kaldo_batch_run(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_BF16X3, gbf))
    torch.cuda.synchronize()
    f0.record(stream)
    kaldo._check(ctx.h, kaldo.kaldo_batch_run(ctx.h, T, sigma, kaldo.KALDO_QUANTUM, kaldo.KALDO_BF16X3, None))
    f1.record(stream)
    torch.cuda.synchronize()
    msbf = f0.elapsed_time(f1)
    ctx.close()
    log(f"batch bf16x3 (first ceil(N_k/{div}) points): {msbf:.1f} ms per launch")
    errbf = 0.0
    for a, b, m in zip(gbf, g64, sub):
        x, y = a[:, :m], b[:, :m]
        on = y > 0
        floor = 1e-6 * np.abs(y).max()
        errbf = max(errbf, float(np.max(np.abs(x[on] - y[on]) / np.maximum(y[on], floor))))
    err = 0.0
    for a, b, m in zip(g32, g64, sub):
        x, y = a[:, :m], b[:, :m]
        on = y > 0
        floor = 1e-6 * np.abs(y).max()
        err = max(err, float(np.max(np.abs(x[on] - y[on]) / np.maximum(y[on], floor))))
    # ---- work accounting (computed first-mode points: one of each pair k, -k)
    pts = [computed_points(c.grid) if share == 1 else shared_points(c.grid, m) for c, m in zip(crystals, share_pts)]
    fa = fb = fc = 0.0
    for c, p in zip(crystals, pts):
        a, b, cc = batch_flops(c, p)
        fa, fb, fc = fa + a, fb + b, fc + cc
    pts64 = sub
    fc64 = sum(batch_flops(c, p)[2] for c, p in zip(crystals, pts64))
    lw = sum(m * c.n_modes for c, m in zip(crystals, share_pts)) * len(T)
    lw64 = sum(m * c.n_modes for c, m in zip(crystals, sub)) * len(T)
    ran = ex / dense if dense else 1.0
    kernel_ms = graph_ms / max(launches, 1)
    # per crystal: workgroup 0's clock over its rounds, against its algorithmic flops
    crystal_rows = []
    for i, c in enumerate(crystals):
        if i in per_crystal:
            f = batch_flops(c, pts[i])[2]
            crystal_rows.append({"crystal": c.name, "ms": per_crystal[i], "tflops": f / (per_crystal[i] * 1e-3) / 1e12,
                                 "frac": f / (per_crystal[i] * 1e-3) / FP32_MFMA_PEAK})
    crystal_rows.sort(key=lambda r: -r["ms"])
    return dict(per_crystal=crystal_rows, phases=phases, crystals=crystals, share=share, share_pts=share_pts, T=T, sigma=sigma, ms=ms, wall=wall, kernel_ms=kernel_ms, ran=ran, ex=ex / steps,
                dense=dense / steps, fa=fa, fb=fb, fc=fc, lw=lw, pts=sum(pts), phonon_s=phonon_s, setup_s=setup_s,
                g32=g32, fp64={"ms_per_launch": ms64, "value": lw64 / (ms64 * 1e-3), "unit": "linewidths/s",
                               "first_mode_points": f"ceil(N_k/{div}) per crystal, {sum(sub)} of "
                                                    f"{sum(c.n_k for c in crystals)}",
                               "gemm_tflops_algorithmic": fc64 / (ms64 * 1e-3) / 1e12,
                               "frac_of_fp64_mfma_peak": fc64 / (ms64 * 1e-3) / FP64_MFMA_PEAK},
                bf16x3={"ms_per_launch": msbf, "value": lw64 / (msbf * 1e-3), "unit": "linewidths/s",
                        "first_mode_points": f"ceil(N_k/{div}) per crystal, the FP64 leg's",
                        "gemm_tflops_algorithmic": fc64 / (msbf * 1e-3) / 1e12,
                        "frac_of_bf16x3_rate": fc64 / (msbf * 1e-3) / (BF16_MFMA_PEAK / 3.0),
                        "gamma_rel_err_vs_fp64": errbf, "speedup_vs_fp64": ms64 / msbf},
                err_fp32_vs_fp64=err)


def run_plain(name, precision, passes=2):
    """One workload on the library's own stream with host outputs: the command
    to run under rocprofv3 counters.  torch initialises the GPU first, as in
    every other run of this file, but hands the library no stream or tensor."""
    import torch
    torch.cuda.init()
    from gen import workload, WORKLOADS
    from paper_2009_01967_amd import kaldo
    w = WORKLOADS[name]
    c = workload(name)
    log(f"{name}: phonons")
    with kaldo.Context(0) as ctx:
        ctx.phonons(c)
        for r in range(passes):
            log(f"{name} {precision} pass {r}: start")
            t0 = time.perf_counter()
            ctx.linewidths(c, T=list(w["T"]), sigma_thz=w["sigma_thz"], precision=precision)
            (ctx.kappa_qhgk if c.n_k == 1 else ctx.kappa_rta)()
            log(f"{name} {precision} pass {r}: {1e3 * (time.perf_counter() - t0):.1f} ms")


def run_next2(steps=3):
    """The variants beside the Gaussian linewidths on the headline workload:
    the FP32 step with the Lorentzian and the triangle delta (same kernels,
    other delta kind), and the FP64 phase space per mode (kaldo_phase_space,
    frequencies only)."""
    import torch
    from gen import workload, WORKLOADS
    from paper_2009_01967_amd import kaldo
    w = WORKLOADS[WORKLOAD]
    c = workload(WORKLOAD)
    T, sigma = list(w["T"]), w["sigma_thz"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    g_d = torch.empty((len(T), c.n_k, c.n_modes), dtype=torch.float64, device=dev)
    out = {"workload": WORKLOAD, "steps": steps}
    with kaldo.Context(0, stream.cuda_stream) as ctx:
        ctx.phonons(c)
        ctx.linewidths(c, T=T, sigma_thz=sigma, precision="fp32", want_host=False)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        lw = c.n_k * c.n_modes * len(T)
        for kind in ("lorentz", "triangle"):
            ms = timed(lambda: kaldo._check(ctx.h, kaldo.kaldo_linewidths(
                ctx.h, None, T, sigma, stats=kaldo.KALDO_QUANTUM, precision=kaldo.KALDO_FP32, gamma_out=g_d,
                delta=kaldo.DELTAS[kind])))
            out[f"linewidths_fp32_{kind}"] = {"ms_per_call": ms, "value": lw / (ms * 1e-3), "unit": "linewidths/s"}
            log(f"next2: FP32 linewidths with the {kind} delta: {ms:.2f} ms")
        ms = timed(lambda: kaldo._check(ctx.h, kaldo.kaldo_phase_space(
            ctx.h, T, sigma, delta=kaldo.KALDO_DELTA_GAUSS, stats=kaldo.KALDO_QUANTUM, g_out=g_d)))
        out["phase_space_fp64_gauss"] = {"ms_per_call": ms, "value": lw / (ms * 1e-3), "unit": "modes/s",
                                         "triples_per_s": c.n_k * c.n_k * c.n_modes ** 3 / (ms * 1e-3)}
        log(f"next2: FP64 phase space: {ms:.2f} ms")
    return out


def run_next1(methods=("inverse", "self-consistent"), max_terms=200):
    """The full linearised BTE on the headline workload (kaldo_kappa_bte): the
    FP64 off-diagonal scattering operator of all 24 576 modes at the three
    temperatures, solved by LU on the time-reversal-odd set vectors and by the
    self-consistent series, beside the RTA of the same linewidths."""
    import torch
    from gen import workload, WORKLOADS
    from paper_2009_01967_amd import kaldo
    w = WORKLOADS[WORKLOAD]
    c = workload(WORKLOAD)
    T, sigma = list(w["T"]), w["sigma_thz"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    out = {"workload": WORKLOAD, "T_K": T, "operator": "fp64"}
    with kaldo.Context(0, stream.cuda_stream) as ctx:
        ctx.phonons(c)
        ctx.linewidths(c, T=T, sigma_thz=sigma, precision="fp64", want_host=False)
        k_rta = ctx.kappa_rta()
        out["kappa_rta_diag"] = [list(np.diag(k)) for k in k_rta]
        for m in methods:
            kaldo.kaldo_profile_enable(ctx.h, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k, terms, ok = ctx.kappa_bte(m, max_terms=max_terms, tol=1e-12)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            kern = {}
            for name in ("bte_scatter", "bte_operator", "bte_solve"):
                tot, cnt = kaldo.kaldo_profile_read(ctx.h, name)
                kern[name] = tot
            kaldo.kaldo_profile_enable(ctx.h, False)
            out[m] = {"ms_per_call": wall, "kernels_ms": kern, "terms": terms, "converged": ok,
                      "kappa_diag": [list(np.diag(x)) for x in k],
                      "kappa_over_rta_xx": [float(x[0, 0] / r[0, 0]) for x, r in zip(k, k_rta)]}
            log(f"next1 {m}: {wall:.1f} ms, terms {terms}, converged {ok}, kernels {kern}, "
                f"kappa/rta {out[m]['kappa_over_rta_xx']}")
    return out


def run_section(flags, key):
    """One optional section of the benchmark (the many-branch MFMA workloads)
    in a child process, so that a failure there costs that section only.  The
    child's progress goes to this process's stderr; its JSON line is parsed.
    Returns (value, None) or (None, reason)."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--no-main"] + flags
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=None, text=True, timeout=1800, cwd=ROOT)
    except subprocess.TimeoutExpired:
        return None, "section timed out"
    lines = [ln for ln in r.stdout.splitlines() if ln.strip().startswith("{")]
    if r.returncode != 0 or not lines:
        return None, f"section exited with status {r.returncode}"
    return json.loads(lines[-1]).get(key), None


def measured_peaks():
    """Attainable rates of the units the kernels use, from register-only MFMA /
    FMA loops and a 1 GiB streaming copy (libpeaks.so), beside the published
    peaks that the roofline fractions use."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2009_01967_amd", "libpeaks.so"))
    for name in ("mi355x_peak_mfma_bf16", "mi355x_peak_mfma_f32", "mi355x_peak_mfma_f64"):
        getattr(lib, name).restype = ctypes.c_double
    lib.mi355x_peak_valu.restype = ctypes.c_double
    lib.mi355x_peak_valu.argtypes = [ctypes.c_int]
    lib.mi355x_peak_hbm.restype = ctypes.c_double
    lib.mi355x_peak_hbm.argtypes = [ctypes.c_size_t]
    out = {"mfma_bf16_tflops": lib.mi355x_peak_mfma_bf16() / 1e12,
           "mfma_f32_tflops": lib.mi355x_peak_mfma_f32() / 1e12,
           "mfma_f64_tflops": lib.mi355x_peak_mfma_f64() / 1e12,
           "valu_f32_tflops_nonpacked": lib.mi355x_peak_valu(0) / 1e12,
           "valu_f64_tflops": lib.mi355x_peak_valu(1) / 1e12,
           "hbm_copy_gbps": lib.mi355x_peak_hbm(1 << 30) / 1e9,
           "published": {"mfma_bf16_tflops": 2500.0, "mfma_f32_tflops": 157.3, "mfma_f64_tflops": 78.6,
                         "valu_f32_tflops": 157.3, "valu_f64_tflops": 78.6, "hbm_gbps": 8000.0}}
    log(f"measured peaks: {out}")
    return out


def c2_section(r):
    """The few-branch workload's JSON (the VALU kernel's roofline)."""
    nk, n, nd, nT = r["nk"], r["n"], r["nd"], len(r["T"])
    lw = nk * n * nT
    npts = computed_points(r["c"].grid)
    f_b, f_c = algorithmic_flops(nk, n, nd, npts)
    proj32 = r["kern32"]["project"]["avg_ms"]
    proj64 = r["kern64"]["project"]["avg_ms"]
    return {
        "workload": WORKLOAD, "n_k": nk, "n_modes": n, "n_T": nT, "T_K": r["T"], "sigma_thz": r["sigma"],
        "fc3_blocks": int(len(r["c"].fc3_i)), "n_delta": nd,
        "step": "kaldo_phonons + kaldo_linewidths + kaldo_kappa_rta on resident inputs",
        "fp32": {"ms_per_step": r["ms32"], "value": lw / (r["ms32"] * 1e-3), "unit": "linewidths/s",
                 "projection_tflops": (f_b + f_c) / (r["ms32"] * 1e-3) / 1e12},
        "fp64": {"ms_per_step": r["ms64"], "value": lw / (r["ms64"] * 1e-3), "unit": "linewidths/s",
                 "projection_tflops": (f_b + f_c) / (r["ms64"] * 1e-3) / 1e12, "project_kernel_ms": proj64},
        "speedup_fp32_vs_fp64": r["ms64"] / r["ms32"],
        "kernels_ms": {k: v["avg_ms"] for k, v in r["kern32"].items()},
        "roofline": {
            "bound": "alu", "kernel": "k_project_small<float,6,3,true,0>",
            "achieved": (f_b + f_c) / (proj32 * 1e-3) / 1e12 if proj32 else None,
            "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": (f_b + f_c) / (proj32 * 1e-3) / FP32_VECTOR_PEAK if proj32 else None,
            "traffic": C2_TRAFFIC["fetch_bytes"] + C2_TRAFFIC["write_bytes"] if C2_TRAFFIC else None,
            "traffic_unit": "bytes per launch (HBM, calibrated FETCH_SIZE + WRITE_SIZE)",
            "intermediate_bytes": intermediate_bytes(nk, n, nd, nT, npts),
            "algorithmic_bytes": survey_algorithmic_bytes(r["c"], nT),
            "flops_per_launch": f_b + f_c,
            "first_mode_points_computed": npts,
            "flops_executed_per_launch": f_b * (nd - r["npair"]) / nd + f_c,
            "executed_frac": ((f_b * (nd - r["npair"]) / nd + f_c) / (proj32 * 1e-3) / FP32_VECTOR_PEAK
                              if proj32 else None),
            "delta_pairs": r["npair"],
        },
    }


def cpu_baseline_batch(b, budget_s=20.0):
    """The FP64 oracle on the host on a sample of the batch: first-mode points
    of the 36-branch crystal (12 atoms on 9^3) until the budget is spent; the
    whole batch's time is extrapolated with each crystal's cost per point
    (16 N_k n^4, the oracle evaluates every point) and compared with the
    library's FP32 values at the sampled points."""
    from oracle import phonons as P, anharmonic as A
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    crystals, T, sigma = b["crystals"], b["T"], b["sigma"]
    ci = min(range(len(crystals)), key=lambda i: (abs(crystals[i].n_modes - 36), crystals[i].n_k))
    c = crystals[ci]
    ph = P.phonons(c, velocities=False)
    t0 = time.perf_counter()
    done, ref = [], []
    for k in (1, 2, 3, 5, 7, 11, 13):
        ref.append(A.linewidths(c, ph, T, sigma, k_subset=[k])[:, 0])
        done.append(k)
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    per_flop = el / (len(done) * 16.0 * c.n_k * c.n_modes ** 4)
    full_s = per_flop * sum(16.0 * x.n_k * x.n_k * x.n_modes ** 4 for x in crystals)
    g = np.stack(ref, axis=1)
    mask = ph.mask[done]
    gs = b["g32"][ci][:, done]
    floor = 1e-6 * np.abs(g[:, mask]).max()
    err = float(np.max(np.abs(gs[:, mask] - g[:, mask]) / np.maximum(np.abs(g[:, mask]), floor)))
    return {"value": b["lw"] / full_s, "unit": "linewidths/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(done)} first-mode points of {c.name} ({c.n_modes} branches, {c.n_k} points) in "
                      f"{el:.1f} s, numpy float64 on {os.cpu_count()} host cores; the 32-crystal batch "
                      f"extrapolated by 16 N_k^2 n^4 per crystal to {full_s:.3e} s"}, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed launches of the batch graph (headline)")
    ap.add_argument("--warmup", type=int, default=0, help="untimed launches of the batch graph before timing")
    ap.add_argument("--batch-share", type=int, default=1,
                    help="time the batch on the first ceil(N_k / S) first-mode points of each crystal (default 1: "
                         "every point, the headline workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-mfma", action="store_true", help="skip the many-branch MFMA workloads")
    ap.add_argument("--no-c2", action="store_true", help="skip the few-branch diamond workload and its variants")
    ap.add_argument("--no-next2", action="store_true",
                    help="skip the Lorentzian/triangle linewidths and the phase space on the diamond workload")
    ap.add_argument("--no-next1", action="store_true",
                    help="skip the full linearised BTE (inverse and self-consistent) on the diamond workload")
    ap.add_argument("--peaks", action="store_true", help="only measure the attainable unit peaks")
    ap.add_argument("--plain", metavar="WORKLOAD", help="run one workload through the library alone "
                    "(torch initialises the GPU but hands the library no stream or tensor; for rocprofv3 "
                    "counters) with --precision, then exit")
    ap.add_argument("--precision", default="bf16x3")
    ap.add_argument("--no-main", action="store_true",
                    help="only the many-branch workloads (prints their JSON; for profiling and the child section)")
    ap.add_argument("--c2-only", action="store_true",
                    help="only the few-branch diamond workload (prints its JSON section; for profiling), with "
                         "--steps timed FP32 steps after --warmup")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): it measures one GPU's share of "
              f"the path; a sharded run would give each GPU a range of first-mode points "
              f"(kaldo_set_k_range)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes, "copies": 3}}))
        return
    if args.plain:
        run_plain(args.plain, args.precision)
        return
    if args.peaks:
        import torch
        torch.cuda.init()
        print(json.dumps({"measured_peaks": measured_peaks()}))
        return
    if args.c2_only:
        import torch
        torch.cuda.init()
        print(json.dumps({"fewbranch_c2": c2_section(run_c2(steps=max(args.steps, 2), warmup=max(args.warmup, 1)))}))
        return
    if args.no_main:
        print(json.dumps({"mfma_paths": [run_mfma(name, steps=2, warmup=1) for name in MFMA_WORKLOADS]}))
        return
    # the many-branch workloads run first, in a child process started before
    # this process touches the GPU
    sections = {}
    if not args.no_mfma:
        sections["mfma_paths"] = run_section([], "mfma_paths")
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    b = run_batch_headline(args.steps, args.warmup, share=args.batch_share)
    value = b["lw"] / (b["ms"] * 1e-3)
    kms = b["kernel_ms"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "linewidths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD + ("" if b["share"] == 1 else f", first ceil(N_k/{b['share']}) points"),
                   "crystals": len(b["crystals"]),
                   "modes": int(sum(m * c.n_modes for c, m in zip(b["crystals"], b["share_pts"]))), "T_K": b["T"],
                   "sigma_thz": b["sigma"], "projection": "fp32", "accumulation": "fp64",
                   "first_mode_points_computed": b["pts"],
                   "launch": "one HIP graph launch: one persistent kernel over the cost-sorted rounds"},
        "wall_ms_per_step": b["wall"],
        "setup_s": {"phonons": b["phonon_s"], "plan_and_capture": b["setup_s"]},
        "projection_tflops": b["fc"] / (b["ms"] * 1e-3) / 1e12,
        "roofline": {
            "bound": "mfma", "kernel": "k_batch_persistent<1,1> (FP32, one temperature)",
            "achieved": b["fc"] / (kms * 1e-3) / 1e12, "peak": FP32_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": b["fc"] / (kms * 1e-3) / FP32_MFMA_PEAK,
            "traffic": (HEADLINE_TRAFFIC["fetch_bytes"] + HEADLINE_TRAFFIC["write_bytes"]
                        if HEADLINE_TRAFFIC and b["share"] == 1 else None),
            "traffic_unit": "bytes per launch (HBM, calibrated FETCH_SIZE + WRITE_SIZE)",
            "basis": "algorithmic GEMM flops F_C = 16 N_k n^4 per computed first-mode point, summed over the "
                     "crystals, per launch, over the launch's duration (library events on the stream)",
            "flops_per_launch": b["fc"],
            "step_a_b_flops_per_launch": b["fa"] + b["fb"],
            "useful_frac": b["fc"] * b["ran"] / (kms * 1e-3) / FP32_MFMA_PEAK,
            "tiles_skipped_frac": 1.0 - b["ran"],
            "mfma_tflops_issued": b["ex"] / (kms * 1e-3) / 1e12,
            "kernel_ms": kms,
            "phases_ms": b["phases"],
            "per_crystal": b["per_crystal"],
        },
        "fp64": b["fp64"],
        "bf16x3": b["bf16x3"],
        "speedup_fp32_vs_fp64_per_flop": (b["fc"] / b["ms"]) / (b["fp64"]["gemm_tflops_algorithmic"] * 1e9),
        "gamma_rel_err_fp32_vs_fp64": b["err_fp32_vs_fp64"],
    }
    if not args.no_c2:
        r = run_c2()
        out["fewbranch_c2"] = c2_section(r)
        if not args.no_next2:
            out["next2"] = run_next2()
        if not args.no_next1:
            out["next1"] = run_next1()
    for key, (val, why) in sections.items():
        if val is not None:
            out[key] = val
        else:
            out[key + "_error"] = why
    out["measured_peaks"] = measured_peaks()
    if not args.no_cpu:
        base, err = cpu_baseline_batch(b)
        out["cpu_baseline"] = base
        out["err_vs_oracle"] = {"fp32": err}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
