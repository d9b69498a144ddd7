"""One GPU's share of a run sharded over first-mode grid points
(kaldo_set_k_range, kaldo_batch_set_k_range): the linewidths of a shard equal
those of the full run on its points, are 0 elsewhere, and the RTA
conductivities of the shards add up to the full one.  Few-branch kernel,
crystal GEMMs and the batch graph; argument errors."""

import sys

import numpy as np
import pytest

from gen import random_crystal, workload, batch_crystals

pytestmark = pytest.mark.gpu

T = [300.0, 600.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _shards(c, precision, cuts, sigma=0.3):
    from paper_2009_01967_amd import kaldo
    with kaldo.Context(0) as ctx:
        kaldo._check(ctx.h, kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_FIXED))
        ctx.phonons(c)
        g_full = ctx.linewidths(c, T=T, sigma_thz=sigma, precision=precision)
        k_full = ctx.kappa_rta()
        parts = []
        for k0, k1 in zip(cuts[:-1], cuts[1:]):
            ctx.set_k_range(k0, k1)
            g = ctx.linewidths(None, T=T, sigma_thz=sigma, precision=precision)
            parts.append((k0, k1, g, ctx.kappa_rta()))
    return g_full, k_full, parts


@pytest.mark.parametrize("name,precision", [("diamond-4x4x4", "fp64"), ("diamond-4x4x4", "fp32"),
                                            ("four-atom-3x3x2", "fp64"), ("four-atom-3x3x2", "bf16x3")])
def test_shards_reproduce_the_full_run(name, precision):
    if name == "diamond-4x4x4":
        c = workload("diamond-2at-4x4x4-shell1")
        cuts = [0, 17, 40, 64]
    else:
        c = random_crystal(4, 3, np.random.default_rng(404)).with_grid((3, 3, 2))
        cuts = [0, 5, 18]
    _say(f"case: shards {cuts} of {name}, {precision}")
    g_full, k_full, parts = _shards(c, precision, cuts)
    k_sum = np.zeros_like(k_full)
    for k0, k1, g, kap in parts:
        inside = np.zeros(c.n_k, bool)
        inside[k0:k1] = True
        assert np.all(g[:, ~inside] == 0.0)
        err = float(np.max(np.abs(g[:, inside] - g_full[:, inside])) / np.abs(g_full).max())
        _say(f"  [{k0}, {k1}): gamma difference {err:.2e}")
        assert err < 1e-13, err
        k_sum += kap
    rel = float(np.linalg.norm(k_sum - k_full) / np.linalg.norm(k_full))
    _say(f"  summed kappa vs full: {rel:.2e}")
    assert rel < 1e-12, rel


def test_batch_shards():
    from paper_2009_01967_amd import kaldo
    crystals = batch_crystals(count=3, n_range=(2, 6), g_range=(3, 4))
    _say("case: batch with per-crystal k ranges")
    with kaldo.Context(0) as ctx:
        kaldo._check(ctx.h, kaldo.kaldo_set_tuning(ctx.h, kaldo.KALDO_TUNE_FIXED))
        for c in crystals:
            ctx.batch_add(c)
        full = ctx.batch_run(T=T, sigma_thz=0.3, precision="fp32")
        ranges = [(c.n_k // 3, c.n_k // 3 + 5) for c in crystals]
        for i, (k0, k1) in enumerate(ranges):
            ctx.batch_set_k_range(i, k0, k1)
        part = ctx.batch_run(T=T, sigma_thz=0.3, precision="fp32")
        again = ctx.batch_run(T=T, sigma_thz=0.3, precision="fp32")
    for c, (k0, k1), gf, gp, ga in zip(crystals, ranges, full, part, again):
        assert np.array_equal(gp, ga)
        inside = np.zeros(c.n_k, bool)
        inside[k0:k1] = True
        assert np.all(gp[:, ~inside] == 0.0)
        err = float(np.max(np.abs(gp[:, inside] - gf[:, inside])) / np.abs(gf).max())
        _say(f"  {c.n_atoms} atoms, grid {c.grid}, [{k0}, {k1}): {err:.2e}")
        assert err < 1e-13, err


def test_k_range_errors():
    from paper_2009_01967_amd import kaldo
    c = workload("diamond-2at-4x4x4-shell1")
    _say("case: k range errors")
    with kaldo.Context(0) as ctx:
        assert kaldo.kaldo_set_k_range(ctx.h, -1, 5) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_set_k_range(ctx.h, 5, 5) == kaldo.KALDO_EINVAL
        ctx.phonons(c)
        ctx.set_k_range(64, 100)          # beyond the 64 points: nothing to compute
        st = kaldo.kaldo_linewidths(ctx.h, kaldo.make_fc3(c.fc3_i, c.fc3_j, c.fc3_l, c.fc3_R1, c.fc3_R2,
                                                          c.fc3_val, kaldo._Keep()),
                                    T, 0.3, kaldo.KALDO_QUANTUM, kaldo.KALDO_FP64, None)
        assert st == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_batch_set_k_range(ctx.h, 0, 0, 4) == kaldo.KALDO_EINVAL   # empty batch
        ctx.batch_add(c)
        assert kaldo.kaldo_batch_set_k_range(ctx.h, 0, 64, 70) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_batch_set_k_range(ctx.h, 1, 0, 4) == kaldo.KALDO_EINVAL
        assert kaldo.kaldo_batch_set_k_range(ctx.h, 0, 0, 4) == kaldo.KALDO_OK
