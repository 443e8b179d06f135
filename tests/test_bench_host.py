"""Host-side logic of bench.py: the counter-measured HBM traffic is reported
only for the kernel sources and the bench job it was measured on."""
import json
import os

import bench


def _tree(tmp_path, monkeypatch, entry):
    csrc = tmp_path / "paper_1210_0748_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("// kernel source\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    t = {"source_digest": bench.kernel_source_digest(), "kernels": {"signature": entry}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(t))
    return csrc


def test_traffic_for_the_measured_job(tmp_path, monkeypatch):
    _tree(tmp_path, monkeypatch, {"workload": "powerlaw-10M-100M", "early_stop": True, "k_cap": 10,
                                  "bytes_per_launch": 1234.0})
    assert bench.load_traffic("signature", "powerlaw-10M-100M", True, 10) == 1234.0
    # another job: its launches average differently
    assert bench.load_traffic("signature", "powerlaw-10M-100M", False, 10) is None
    assert bench.load_traffic("signature", "powerlaw-100M-1B", True, 10) is None
    assert bench.load_traffic("signature", "powerlaw-10M-100M", True, 5) is None
    assert bench.load_traffic("order", "powerlaw-10M-100M", True, 10) is None


def test_traffic_dropped_when_sources_change(tmp_path, monkeypatch):
    csrc = _tree(tmp_path, monkeypatch, {"workload": "w", "early_stop": True, "k_cap": 10,
                                         "bytes_per_launch": 1.0})
    assert bench.load_traffic("signature", "w", True, 10) == 1.0
    (csrc / "k.hip").write_text("// kernel source, changed\n")
    assert bench.load_traffic("signature", "w", True, 10) is None


def test_no_traffic_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("signature", "w", True, 10) is None


def test_committed_traffic_names_its_job():
    with open(os.path.join(os.path.dirname(bench.__file__), "profiles", "traffic.json")) as f:
        t = json.load(f)
    e = t["kernels"]["signature"]
    assert e["workload"] == "powerlaw-10M-100M" and e["early_stop"] is True and e["k_cap"] == 10
