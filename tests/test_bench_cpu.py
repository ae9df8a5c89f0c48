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


def test_cpu_baseline_runs_the_oracle_on_the_workload_sample():
    from paper_2604_14411_amd import synth
    from paper_2604_14411_amd.synth.configs import WORKLOADS, Workload

    b = _bench()
    w = Workload("tiny", 64, 400, lambda: synth.random_snn(3000, 20.0, 5), "tiny",
                 lambda: synth.random_snn(300, 10.0, 5), "a random SNN of 300 nodes",
                 (lambda: synth.random_snn(100, 8.0, 5), "a random SNN of 100 nodes"))
    for mlp in (None, synth.random_int_mlp(3)):
        cb = b.cpu_baseline(w, mlp, 2)
        assert cb["kind"] == "oracle" and cb["cores"] == 2 and cb["value"] > 0
        assert cb["proposal"] == ("plain" if mlp is None else "learned")
        assert cb["sample_pins"] == synth.random_snn(300, 10.0, 5).n_pins
        assert cb["single_thread"]["cores"] == 1 and cb["single_thread"]["value"] > 0
        assert cb["nproc"] >= 1 and cb["cpu_model"]
    # every benchmark workload names a sample of its own generator
    for name, wl in WORKLOADS.items():
        assert wl.sample is not None and wl.sample_note, name
