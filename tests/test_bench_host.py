"""Host-side parts of bench.py: the one-GPU contract and the traffic figure
read from the committed counter summary only while the kernel sources it
was measured on are unchanged."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _profile(tmp_path, sha, value="4.87152e+09"):
    p = tmp_path / "traffic.md"
    p.write_text(f"# summary\n\ntraffic_bytes_per_launch: {value}\nkernel_source_sha256: {sha}\n")
    return p


def test_traffic_read_while_sources_match(tmp_path, monkeypatch):
    p = _profile(tmp_path, bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(p))
    assert bench.profiled_traffic() == 4.87152e9


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    p = _profile(tmp_path, "0" * 64)
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(p))
    assert bench.profiled_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic() is None


def test_source_hash_covers_the_kernel_files():
    # every file the interaction kernel is built from is part of the hash
    for f in ("g6mi_kernels.hip", "g6mi_device.h", "g6mi_internal.h", "g6mi_spatial.hip"):
        assert any(k.endswith(f) for k in bench.KERNEL_SOURCES), f
    for k in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, k)), k
