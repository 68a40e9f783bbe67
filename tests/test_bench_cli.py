"""The benchmark's command-line contract and its traffic-record lookup (CPU)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    out = json.loads(p.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_sources_digest_is_stable_and_short():
    d = bench.sources_digest()
    assert d == bench.sources_digest()
    assert len(d) == 16 and all(ch in "0123456789abcdef" for ch in d)


def test_traffic_record_needs_the_current_digest(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    d = bench.sources_digest()
    (prof / "solve_kernels_g20_3d64.md").write_text(
        "text\n"
        f"traffic-record: kernel=k_half<float, 2, 1> bytes_per_launch=123 sources={d}\n"
        "traffic-record: kernel=k_resid<float, 2, 1> bytes_per_launch=456 sources=0000000000000000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the digest is computed over the sources under ROOT: keep the real one
    monkeypatch.setattr(bench, "sources_digest", lambda: d)
    assert bench.recorded_traffic("k_half<float, 2, 1>") == 123
    assert bench.recorded_traffic("k_resid<float, 2, 1>") is None   # stale record
    assert bench.recorded_traffic("k_fhalf0<float, 2, 1>") is None  # no record


def test_error_against_is_per_segment():
    import numpy as np
    ref = np.concatenate([np.full(4, 10.0), np.full(4, 1e-3), np.full(4, 2.0)])
    x = ref.copy()
    x[5] += 1e-9          # segment 1: max 1e-3, so 1e-6 of its scale
    e = bench.error_against(x, ref, 1)
    assert abs(e["max_abs_over_segment_max"] - 1e-6) < 1e-12
    assert 0 < e["rel_2norm"] < 1e-9
