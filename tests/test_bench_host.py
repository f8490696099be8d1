"""Host logic of bench.py (no GPU): the one-GPU contract and the HBM-traffic
figure, which is taken from a committed counter summary only while that
summary names the current kernel source."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _summary(tmp_path, digest, nbytes="4.3449e+10"):
    p = tmp_path / "traffic.md"
    p.write_text(f"hbm_bytes_per_launch: {nbytes}\n\nkernel source sha256[:16]: {digest}\n")
    return str(p)


def test_traffic_read_while_the_source_matches(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _summary(tmp_path, bench._source_hash()))
    assert bench.measured_traffic() == 4.3449e10


def test_traffic_dropped_once_the_source_changed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _summary(tmp_path, "0123456789abcdef"))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None
