"""Host-side checks of the benchmark contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_closed_form():
    """4 nnz (col) + 8 (N+1) (row pointers) + 4 N (degree scale) + 3 * 4 k N
    (read X_m, read X_{m-1}, write X_{m+1}) [+ 8 N with per-node moments]."""
    n, nnz, k = 1_050_000, 10_099_970, 64
    want = 4 * nnz + 8 * (n + 1) + 4 * n + 12 * k * n + 8 * n
    assert bench.algorithmic_bytes(n, nnz, k, True) == want == 867_799_888
    assert bench.algorithmic_bytes(n, nnz, k, False, state_bytes=8) == 4 * nnz + 8 * (n + 1) + 4 * n + 24 * k * n
    assert bench.algorithmic_bytes(n, nnz, k, False, own_row=True) == 4 * nnz + 8 * (n + 1) + 4 * n + 16 * k * n


@pytest.mark.parametrize("workload", ["ba1m_twins", "rmat27"])
def test_traffic_records_match_the_kernel_sources(workload):
    """The committed counter records were taken on the kernel sources as they
    are: otherwise the benchmark would report no traffic."""
    t = bench.profiled_traffic(workload)
    assert t is not None and t > 0
