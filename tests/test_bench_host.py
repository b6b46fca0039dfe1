"""Host-side logic of bench.py (no GPU): the one-GPU guard and the lookup of the
committed HBM-traffic figures, which must apply only to the profiled workload and
to the kernel sources the counters were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""                                  # no JSON line


def test_traffic_figures_follow_the_summary():
    text = open(os.path.join(ROOT, "profiles", "dstage_counters_mw_L2048_spin0.md")).read()
    want = {}
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic_bytes":
            want[parts[1]] = float(parts[2])
    assert set(want) == {"k_dstage_inv", "k_dstage_fwd"}
    for k, v in want.items():
        assert 1e8 < v < 1e11
        if f"kernels source sha256 (first 16 hex): {bench.kernel_source_sha()}" in text:
            assert bench.measured_traffic(k, 2048, 0) == v
        else:                                              # summary taken on other sources
            assert bench.measured_traffic(k, 2048, 0) is None


def test_traffic_is_null_off_the_profiled_workload_or_sources(monkeypatch):
    for L, spin in [(1024, 0), (2048, 2), (4096, 0)]:
        assert bench.measured_traffic("k_dstage_inv", L, spin) is None
    assert bench.measured_traffic("k_no_such_kernel", 2048, 0) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0000000000000000")
    assert bench.measured_traffic("k_dstage_inv", 2048, 0) is None
    assert bench.measured_traffic("k_dstage_fwd", 2048, 0) is None


def test_source_hash_covers_every_sweep_source():
    h = bench.kernel_source_sha()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.kernel_source_sha() == h                  # deterministic
