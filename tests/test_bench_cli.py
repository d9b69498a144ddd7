"""Host-side behaviour of bench.py that needs no GPU: more than one GPU is
refused before anything touches a device, with a message that says so."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_flops_of_the_headline_workload():
    sys.path.insert(0, ROOT)
    import bench
    # diamond 16x16x16: 4096 grid points, 6 modes, 25 cell differences
    f_b, f_c = bench.algorithmic_flops(4096, 6, 25)
    assert f_b == 8.0 * 4096 ** 2 * 25 * 6 ** 3
    assert f_c == 16.0 * 4096 ** 2 * 6 ** 4
    assert abs((f_b + f_c) - 1.0727e12) / 1.0727e12 < 1e-3


def test_failed_section_is_reported_not_raised():
    # a child that exits before touching a GPU (more than one GPU asked for)
    sys.path.insert(0, ROOT)
    import bench
    val, why = bench.run_section(["--gpus", "2"], "mfma_paths")
    assert val is None
    assert "status 2" in why
