"""Host logic of bench.py's HBM-traffic record: the counter record under
profiles/ is used only for the sources and launch shape it was taken on, and its scaling by
the copy calibration is the one documented there."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record(tmp_path, sha, **over):
    r = {"kernel": "k_eloc_lowrank", "workload": "c3", "walkers": 8192, "prec": "f16x2", "slices": 24,
         "src_sha1": sha,
         "fetch_kib": 1000.0, "write_kib": 300.0, "copy_fetch_kib": 524288.0, "copy_write_kib": 1048576.0}
    r.update(over)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x_traffic.md").write_text("# summary\n\ntraffic-record: " + json.dumps(r) + "\n")
    return tmp_path


def test_record_scaled_by_copy_calibration(tmp_path, monkeypatch):
    root = _record(tmp_path, "a" * 40)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "kernel_src_sha1", lambda: "a" * 40)
    tr = bench.traffic_record("c3", 8192, "f16x2", 24)
    assert tr is not None
    # FETCH_SIZE read 512 MiB for a 1 GiB copy: factor 2; WRITE_SIZE exact
    assert tr["fetch_bytes"] == pytest.approx(1000.0 * 1024 * 2.0)
    assert tr["write_bytes"] == pytest.approx(300.0 * 1024)
    assert tr["bytes"] == pytest.approx(tr["fetch_bytes"] + tr["write_bytes"])


def test_record_ignored_for_other_sources_or_workloads(tmp_path, monkeypatch):
    root = _record(tmp_path, "0" * 40)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "kernel_src_sha1", lambda: "1" * 40)
    assert bench.traffic_record("c3", 8192, "f16x2", 24) is None
    monkeypatch.setattr(bench, "kernel_src_sha1", lambda: "0" * 40)
    assert bench.traffic_record("c3", 8192, "f16x2", 24) is not None
    assert bench.traffic_record("c3", 4096, "f16x2", 24) is None
    assert bench.traffic_record("c3", 8192, "bf16x3", 24) is None
    # a record taken at another launch shape does not describe this launch
    assert bench.traffic_record("c3", 8192, "f16x2", 32) is None


def test_source_hash_covers_every_source_file():
    d = os.path.join(ROOT, "paper_2604_25775_amd", "csrc")
    srcs = [f for f in os.listdir(d) if f.endswith((".hip", ".h", ".cpp"))]
    assert srcs, "no library sources found"
    h1 = bench.kernel_src_sha1()
    assert len(h1) == 40 and h1 == bench.kernel_src_sha1()


def test_record_keyed_by_row_form_limit(tmp_path, monkeypatch):
    root = _record(tmp_path, "a" * 40, row_form_max=8)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "kernel_src_sha1", lambda: "a" * 40)
    assert bench.traffic_record("c3", 8192, "f16x2", 24, 8) is not None
    assert bench.traffic_record("c3", 8192, "f16x2", 24, 16) is None
    # a record without the field was taken at the default limit (16)
    root2 = tmp_path / "r2"
    root2.mkdir()
    _record(root2, "a" * 40)
    monkeypatch.setattr(bench, "ROOT", str(root2))
    assert bench.traffic_record("c3", 8192, "f16x2", 24, 16) is not None
    assert bench.traffic_record("c3", 8192, "f16x2", 24, 0) is None
