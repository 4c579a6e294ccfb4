"""Host-side checks of bench.py (no GPU): the one-GPU contract and the
consistency of its measured-traffic records with the kernel sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_records_match_the_kernel_sources():
    # the HBM bytes bench.py reports were counted on the committed kernels:
    # a kernel change without re-taking the counters turns them to null
    h = bench.kernel_src_hash()
    assert len(bench.MEASURED_TRAFFIC) >= 3
    for key, rec in bench.MEASURED_TRAFFIC.items():
        assert rec["src_sha256"] == h, key
        assert rec["bytes"] > 0

