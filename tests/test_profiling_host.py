"""Host logic of the rocprofv3 summaries: kernel statistics, per-dispatch
counters, the copy-calibrated byte scale and the summary round trip that
bench.py reads its traffic figure from."""
import json

import pytest

from paper_2607_26901_amd import profiling


def _write(path, header, rows):
    path.write_text(",".join(header) + "\n" + "\n".join(",".join(str(c) for c in r) for r in rows) + "\n")
    return str(path)


def test_summary_round_trip(tmp_path):
    stats = _write(tmp_path / "s.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
                   [['"ccfr::k_pairs(ccfr::Scene, int)"', 4, 400000, 100000, 60.0],
                    ["k_fill", 8, 80000, 10000, 12.0], ["k_predict", 2, 8000, 4000, 1.0]])
    cnt = ["Kernel_Name", "Counter_Value"]
    fetch = _write(tmp_path / "f.csv", cnt, [["k_pairs", 1000.0], ["k_pairs", 3000.0], ["k_fill", 10.0]])
    write = _write(tmp_path / "w.csv", cnt, [["k_pairs", 500.0], ["k_pairs", 500.0]])
    occ = _write(tmp_path / "o.csv", cnt, [["k_pairs", 40.0], ["k_pairs", 60.0]])
    # a 1 MiB copy counted as 512 KiB fetched and 1024 KiB written
    cf = _write(tmp_path / "cf.csv", cnt, [["copy", 256.0], ["copy", 512.0]])
    cw = _write(tmp_path / "cw.csv", cnt, [["copy", 1024.0]])
    bench = tmp_path / "b.json"
    bench.write_text(json.dumps({"config": {"iters_per_step": 10, "workload": "w"},
                                 "tuning": {"cell_scale": 0.7, "pair_split": 1, "pair_reuse": 3}}) + "\n")
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    out = tmp_path / "summary.md"
    assert profiling.main(["--stats", stats, "--fetch", fetch, "--write", write, "--copy-fetch", cf,
                           "--copy-write", cw, "--copy-mib", "1", "--occupancy", occ, "--source", str(src),
                           "--bench", str(bench), "--command", "cmd", "--out", str(out)]) == 0
    facts = profiling.read_kernel_summary(str(out))
    assert facts["iterations"] == 20                      # 2 substeps of 10 iterations
    kp = facts["kernels"]["k_pairs"]
    assert kp["calls"] == 4 and kp["avg_us"] == pytest.approx(100.0)
    assert kp["fetch_kib"] == 2000.0 and kp["write_kib"] == 500.0
    assert facts["fetch_scale"] == pytest.approx(2.0) and facts["write_scale"] == pytest.approx(1.0)
    # bytes = KiB counted x bytes per counted KiB
    assert kp["traffic_bytes"] == pytest.approx(2000 * 2048 + 500 * 1024)
    assert kp["occupancy_pct"] == pytest.approx(50.0)
    assert "traffic_bytes" not in facts["kernels"]["k_fill"]      # no WRITE_SIZE for it
    assert facts["sources"] == {str(src): profiling.sha256(str(src))}
    assert facts["knobs"] == profiling.knobs_key({"cell_scale": 0.7, "pair_split": 1, "pair_reuse": 3})
    assert "cmd" in out.read_text()


def test_knobs_key_defaults_and_distinguishes():
    a = profiling.knobs_key({"cell_scale": 0.7, "pair_split": 1})
    assert a == profiling.knobs_key({"cell_scale": 0.7000001, "pair_split": 1, "pair_reuse": 1})
    assert a != profiling.knobs_key({"cell_scale": 0.7, "pair_split": 1, "pair_reuse": 3})
    assert a != profiling.knobs_key({"cell_scale": 0.7, "pair_split": 1, "pair_skin": 2})
