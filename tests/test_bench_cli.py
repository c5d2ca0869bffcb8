"""The benchmark's command-line contract that holds without a GPU: more than one
GPU is refused with a message and a non-zero exit status, a served stream longer
than the length that has run cleanly is refused before any GPU work, and the
profile summaries that the roofline figures come from parse."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_profile_summaries_parse():
    sys.path.insert(0, ROOT)
    import bench
    # both summaries carry the hash of the kernel source they were measured on;
    # when it matches the present source, the figures are used, else they are null
    t, v = bench.measured_traffic(), bench.measured_valu_busy()
    if t is not None:
        assert 1.0e9 < t < 1.0e10
    if v is not None:
        assert 0.0 < v <= 1.0


def test_long_served_streams_are_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "served",
                        "--requests", "201"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    assert "served streams of more than 200 requests are refused" in p.stderr
