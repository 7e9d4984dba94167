"""Host-side checks of bench.py: the one-GPU contract and the counter
profile that the headline's traffic figure comes from."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_profile_matches_the_kernel_sources():
    """The committed S12 counter profile was taken on the current product
    kernel sources, so the bench line carries its measured HBM bytes."""
    import bench
    t = bench.measured_traffic()
    assert t is not None, "profile missing or taken on other kernel sources"
    # counted DRAM bytes lie below the 12 nnz + 16 n model (16-bit column
    # offsets) and above the value stream alone (8 nnz)
    nnz, n = 156365811, 1975509
    assert 8 * nnz < t < 12 * nnz + 16 * n


@pytest.mark.parametrize("flag", ["--only-small-batch", "--only-headline",
                                  "--sweep", "--serving-full"])
def test_single_experiment_modes_are_documented(flag):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and flag in r.stdout
