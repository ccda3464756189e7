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
    """4 nnz (col) + 8 (N+1) (row pointers) + 8 N (probe sign words) + 3 * 4 k N
    (read X_m, read X_{m-1}, write X_{m+1}) [+ 4 N twin-class index when
    filtering] [+ 8 N with per-node moments]; doubling / Lanczos steps read
    the own row (4 k N more) and no sign words."""
    n, nnz, k = 1_050_000, 10_099_970, 64
    want = 4 * nnz + 8 * (n + 1) + 8 * n + 4 * n + 12 * k * n + 8 * n
    assert bench.algorithmic_bytes(n, nnz, k, True, filtered=True) == want == 876_199_888
    assert bench.algorithmic_bytes(n, nnz, k, False, state_bytes=8) == 4 * nnz + 8 * (n + 1) + 8 * n + 24 * k * n
    assert bench.algorithmic_bytes(n, nnz, k, False, own_row=True) == 4 * nnz + 8 * (n + 1) + 16 * k * n


def test_traffic_record_only_for_matching_kernel_sources(tmp_path, monkeypatch):
    """A counter record is used only while the kernel sources it was taken on
    are the ones built; a stale one is ignored (traffic reported as null)."""
    import json
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "paper_1905_09758_amd" / "csrc"
    src.mkdir(parents=True)
    for f in bench.STEP_KERNEL_SOURCES:
        (src / f).write_text("// " + f)
    sha = bench.step_kernel_sha256()
    rec = {"kernel_sources_sha256": sha, "bytes_per_launch": 123}
    (prof / "k_cheb_step_w.md").write_text("x\ntraffic_record: " + json.dumps(rec) + "\n")
    assert bench.profiled_traffic("w") == 123
    (src / bench.STEP_KERNEL_SOURCES[-1]).write_text("// changed")
    assert bench.profiled_traffic("w") is None
    assert bench.profiled_traffic("missing") is None
