"""Host-side behaviour of bench.py that needs no GPU: the one-GPU contract
and the rule that HBM traffic from a committed counter summary is used only
while the headline kernel's sources are unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(tmp_path, sha, traffic=12345):
    rec = {"kernel": "k", "source_sha256": sha, "traffic_bytes": traffic}
    p = tmp_path / "summary.md"
    p.write_text("# summary\n\n<!-- traffic " + json.dumps(rec) + " -->\n")
    return str(p)


def test_traffic_used_only_for_unchanged_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE", _summary(tmp_path, bench.stream_source_sha256()))
    assert bench.measured_traffic() == 12345
    monkeypatch.setattr(bench, "PROFILE", _summary(tmp_path, "0" * 64))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_source_hash_covers_the_kernel_and_its_headers(tmp_path, monkeypatch):
    files = []
    for name in ("a.hip", "b.h"):
        f = tmp_path / name
        f.write_text(name)
        files.append(str(f))
    monkeypatch.setattr(bench, "STREAM_SRCS", files)
    h0 = bench.stream_source_sha256()
    (tmp_path / "b.h").write_text("changed")
    assert bench.stream_source_sha256() != h0
