"""Host-side checks of bench.py (no GPU): the byte model its roofline
reports, the HBM counter table against the kernel sources it was taken on,
and the single-GPU contract of its command line."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_voxel_iteration():
    # x pass: spectrum, strain state and stresses read and written, the
    # history base and p_n, q_n read, the phase id; three axis passes of 36 w
    assert bench.algorithmic_x_bytes(8) == 1025 and bench.algorithmic_x_bytes(4) == 521
    assert sum(bench.algorithmic_bytes_per_voxel(8).values()) == 1889
    assert sum(bench.algorithmic_bytes_per_voxel(4).values()) == 953


def test_measured_traffic_matches_the_kernel_sources():
    """Every counter figure the bench reports was taken on the kernels as
    they stand (bench.py reports traffic null otherwise)."""
    sha = bench.kernel_src_sha1()
    for name, entry in bench.MEASURED_TRAFFIC.items():
        assert entry["src_sha1"] == sha, name
        assert entry["bytes"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
