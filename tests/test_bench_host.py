"""Host-side logic of bench.py (no GPU): the one-GPU contract, and that the
counter-based traffic is only reported for the kernel sources it was
measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_hash_is_stable():
    h = bench.kernel_hash()
    assert len(h) == 16 and h == bench.kernel_hash()


def test_traffic_only_for_matching_sources():
    path = os.path.join(ROOT, "profiles", "traffic_laplace_n1m.json")
    d = json.load(open(path))
    assert bench.read_traffic("laplace_n1m", "fp32c", "0" * 16) is None
    assert bench.read_traffic("no_such_workload", "fp32c", d["kernel_hash"]) is None
    got = bench.read_traffic("laplace_n1m", "fp32c", d["kernel_hash"])
    assert got == d["fp32c"]
    assert bench.read_traffic("laplace_n1m", "fp32c", d["kernel_hash"], field="valu_issue") == \
        d["valu_issue"]["fp32c"]

