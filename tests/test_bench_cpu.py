"""Host logic of bench.py: the measured-traffic lookup (no GPU)."""
import hashlib
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _write(tmp_path, sources):
    d = {"classes": {"seq_events": {"bytes_per_launch": 123.5, "sources": sources}}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(d))
    return str(p)


def test_traffic_reported_while_sources_unchanged(tmp_path, monkeypatch):
    b = _bench()
    rel = "bench.py"
    digest = hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()
    monkeypatch.setattr(b, "TRAFFIC_FILE", _write(tmp_path, {rel: digest}))
    assert b.measured_traffic("seq_events") == pytest.approx(123.5)
    assert b.measured_traffic("sort") is None


def test_traffic_dropped_when_a_source_changed(tmp_path, monkeypatch):
    b = _bench()
    monkeypatch.setattr(b, "TRAFFIC_FILE", _write(tmp_path, {"bench.py": "0" * 64}))
    assert b.measured_traffic("seq_events") is None
    monkeypatch.setattr(b, "TRAFFIC_FILE", _write(tmp_path, {"no/such/file.hip": "0" * 64}))
    assert b.measured_traffic("seq_events") is None


def test_committed_traffic_file_is_well_formed():
    b = _bench()
    d = json.load(open(b.TRAFFIC_FILE))
    cal = d["copy_calibration"]
    assert cal["fetch_scale"] > 0 and cal["write_scale"] > 0
    for cls, e in d["classes"].items():
        assert cls in b.COST
        assert e["bytes_per_launch"] > 0 and e["launches"] > 0
        assert all(os.path.exists(os.path.join(ROOT, rel)) for rel in e["sources"])
