"""The rocprofv3 summary tool on hand-made CSV files: per-kernel statistics,
round split, counter averages, the traffic figure of one kernel (with the
bench job it was read on) and measured GB/s per kernel."""
import csv
import json

from paper_1210_0748_amd import profsum

SIG = "void kb::signature_k<unsigned int, unsigned int>(kb::SigArgs)"
SCAT = "void kb::radix_scatter_k<unsigned int>(unsigned int const*)"


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)
    return str(path)


def _counters(path, name, per_kernel):
    rows = [[k, name, v] for k, vals in per_kernel.items() for v in vals]
    return _write(path, ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_stats_and_gbs(tmp_path, capsys):
    stats = _write(tmp_path / "s.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "MaxNs"],
                   [[SIG, 2, 2000.0, 1000.0, 1500.0], [SCAT, 4, 400.0, 100.0, 120.0]])
    profsum.cmd_stats(stats, 10)
    out = capsys.readouterr().out.splitlines()
    assert out[1].startswith("signature_k<unsigned int, unsigned int>")  # by total time
    assert "all kernels: 0.002 ms" in out[-1]
    # 3000 KiB fetched (x2) + 1000 KiB written (x1) per dispatch in 1000 ns
    fetch = _counters(tmp_path / "f.csv", "FETCH_SIZE", {SIG: [2000.0, 4000.0], SCAT: [10.0]})
    write = _counters(tmp_path / "w.csv", "WRITE_SIZE", {SIG: [1000.0, 1000.0], SCAT: [10.0]})
    scales = tmp_path / "t.json"
    scales.write_text(json.dumps({"fetch_scale": 2.0, "write_scale": 1.0}))
    profsum.cmd_gbs(stats, fetch, write, str(scales), 0)
    lines = capsys.readouterr().out.splitlines()
    sig = [ln for ln in lines if ln.startswith("signature_k")][0].split()
    gbs = (3000.0 * 1024 * 2 + 1000.0 * 1024) / 1000.0
    assert abs(float(sig[-2]) - round(gbs)) <= 1 and abs(float(sig[-1]) - gbs / 8000.0) < 1e-3


def test_rounds_split_at_signature(tmp_path, capsys):
    rows = [[SIG, 0, 10], ["void kb::other_k()", 12, 20], [SIG, 30, 35], ["void kb::other_k()", 40, 50]]
    trace = _write(tmp_path / "k.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    profsum.cmd_rounds(trace)
    out = capsys.readouterr().out.splitlines()
    assert out[1].split()[:2] == ["0", "2"] and out[2].split()[:2] == ["1", "2"]


def test_traffic_records_the_job(tmp_path, capsys):
    fetch = _counters(tmp_path / "f.csv", "FETCH_SIZE", {SIG: [100.0, 300.0]})
    write = _counters(tmp_path / "w.csv", "WRITE_SIZE", {SIG: [50.0, 50.0]})
    # the 1 GiB copy reads as 512 MiB fetched and 1 GiB written
    cf = _counters(tmp_path / "cf.csv", "FETCH_SIZE", {"__amd_rocclr_copyBuffer": [512.0 * 1024]})
    cw = _counters(tmp_path / "cw.csv", "WRITE_SIZE", {"__amd_rocclr_copyBuffer": [1024.0 * 1024]})
    out = tmp_path / "traffic.json"
    profsum.main(["traffic", fetch, "--write", write, "--cal-fetch", cf, "--cal-write", cw,
                  "--kernel", "signature_k", "--name", "signature", "--out", str(out),
                  "--workload", "w1", "--k-cap", "7", "--no-early-stop"])
    capsys.readouterr()
    t = json.loads(out.read_text())
    e = t["kernels"]["signature"]
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert e["fetch_bytes_per_launch"] == 200.0 * 1024 * 2 and e["write_bytes_per_launch"] == 50.0 * 1024
    assert (e["workload"], e["early_stop"], e["k_cap"]) == ("w1", False, 7)
    assert t["source_digest"] == profsum.source_digest()
