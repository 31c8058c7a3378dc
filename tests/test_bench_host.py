"""Host-side checks of bench.py: one GPU only, the traffic record tied to
the kernel sources, and the option surface (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_follows_the_kernel_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    rec = {"w/fp32/k": {"bytes_per_launch": 123.0, "source_hash": h},
           "w/fp32/old": {"bytes_per_launch": 9.0, "source_hash": "0" * 16}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel_source_hash reads ROOT's sources: point it back at the repo's
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.traffic_from_profiles("w", "fp32", "k") == 123.0
    assert bench.traffic_from_profiles("w", "fp32", "old") is None
    assert bench.traffic_from_profiles("w", "fp32", "missing") is None


def test_options_parse():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for opt in ("--op", "--lowrank-phase", "--switch-otf", "--graph",
                "--autotune", "composition", "serving"):
        assert opt in r.stdout
