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
import numpy as np  # noqa: E402
import pytest  # noqa: E402


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



def _brute_candidates(x, L, D, n):
    """Ordered (target, source) pairs with the source's leaf box within one
    box of the target's along every axis, counted once per periodic image
    (shift s in {-1, 0, 1} of an axis below D), self pairs included."""
    L = np.asarray(L, dtype=np.float64)
    n = np.asarray(n)
    b = np.empty(x.shape, dtype=np.int64)
    for i in range(3):
        y = np.mod(x[:, i], L[i]) if i < D else x[:, i]
        b[:, i] = np.minimum(n[i] - 1, np.floor(y * (n[i] / L[i])).astype(np.int64))
    total = 0
    for t in range(len(x)):
        m = np.ones(len(x), dtype=np.int64)
        for i in range(3):
            if i < D:
                m *= sum((np.abs(b[:, i] + s * n[i] - b[t, i]) <= 1).astype(np.int64) for s in (-1, 0, 1))
            else:
                m *= (np.abs(b[:, i] - b[t, i]) <= 1).astype(np.int64)
        total += int(m.sum())
    return total


@pytest.mark.parametrize("D,n", [(3, (4, 5, 3)), (2, (2, 1, 6)), (1, (5, 4, 4)), (0, (3, 6, 2))])
def test_candidate_count_matches_brute_force(D, n):
    from paper_2606_27134_amd import workloads as W
    rng = np.random.default_rng(40 + D)
    L = (1.0, 1.5, 0.75)
    x = rng.random((300, 3)) * np.asarray(L)
    w = W.Workload(name="tiny", kernel="laplace", D=D, L=L, n=n, N=len(x), sigma=0.01, rc=0.05, x=x,
                   rho=np.zeros((len(x), 1)), seed=0)
    assert bench.count_candidates(w) == _brute_candidates(x, L, D, n)
