"""The rocprofv3 summary tools behind profiles/: the HBM traffic record
(counters scaled by what they read for a plain copy of known size), the
FP64 matrix-core summary and the kernel-stats table, on small synthetic files."""
import csv
import json
import os

from paper_1405_2810_amd import profiling


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_record_scales_by_the_copy(tmp_path):
    copy = 256 << 20
    # the calibration copy reads 2 KiB units and writes 1 KiB units
    _write_counters(tmp_path / "cf", [("copyBuffer", "FETCH_SIZE", copy / 2048)] * 3)
    _write_counters(tmp_path / "cw", [("copyBuffer", "WRITE_SIZE", copy / 1024)] * 3)
    _write_counters(tmp_path / "f", [("void lrbms::k_flux<2>(lrbms::Geom)", "FETCH_SIZE", 100.0),
                                      ("void lrbms::k_flux<2>(lrbms::Geom)", "FETCH_SIZE", 300.0)])
    _write_counters(tmp_path / "w", [("void lrbms::k_flux<2>(lrbms::Geom)", "WRITE_SIZE", 50.0),
                                      ("void lrbms::k_flux<2>(lrbms::Geom)", "WRITE_SIZE", 50.0)])
    out_json, out_txt = tmp_path / "t.json", tmp_path / "t.txt"
    profiling.main(["traffic", "wl", str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                    str(tmp_path / "cw"), "2", str(out_json), str(out_txt), "cmd"])
    rec = json.load(open(out_json))["wl"]["k_flux"]
    assert rec["fetch_bytes_per_launch"] == 200.0 * 2048
    assert rec["write_bytes_per_launch"] == 50.0 * 1024
    assert rec["launches"] == 2
    assert rec["source_sha"] == profiling.source_sha("k_flux")


def test_mfma_summary(tmp_path):
    _write_counters(tmp_path / "m", [("void lrbms::k_asm_box<2, 32>(lrbms::Geom)",
                                      "SQ_INSTS_VALU_MFMA_MOPS_F64", 1.0e6)] * 4)
    stats = tmp_path / "s"
    os.makedirs(stats)
    with open(stats / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                          "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void lrbms::k_asm_box<2, 32>(lrbms::Geom)", "Calls": 4,
                    "TotalDurationNs": 4 * 51200, "AverageNs": 51200, "Percentage": 100})
    out = tmp_path / "mfma.txt"
    profiling.main(["mfma", str(tmp_path / "m"), str(stats / "run_kernel_stats.csv"), "t",
                    str(out), "cmd"])
    line = [l for l in open(out) if l.startswith("k_asm_box")][0].split()
    # 1e6 x 512 flops per launch over 51.2 us = 10 TFLOP/s, 12.7 % of 78.6
    assert line[1] == "4" and float(line[2]) == 512.0 and float(line[4]) == 10.0
    assert line[5] == "12.72%"


def test_kernel_stats_table(tmp_path):
    """The kernel-stats summary: the title and command lines, then one row
    per kernel with short names, sorted by total time, in ms and us."""
    stats = tmp_path / "s"
    os.makedirs(stats)
    with open(stats / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                          "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void lrbms::k_flux<2>(lrbms::Geom)", "Calls": 10,
                    "TotalDurationNs": 50000, "AverageNs": 5000, "Percentage": 20})
        w.writerow({"Name": "void lrbms::k_front_step(lrbms::StepItem const*)", "Calls": 8,
                    "TotalDurationNs": 200000, "AverageNs": 25000, "Percentage": 80})
    out = tmp_path / "stats.txt"
    profiling.main(["stats", str(stats / "run_kernel_stats.csv"), "title line", "the command",
                    str(out)])
    lines = open(out).read().splitlines()
    assert lines[0] == "# title line" and lines[1] == "# command: the command"
    rows = [l.split() for l in lines[3:]]
    assert [r[0] for r in rows] == ["k_front_step", "k_flux"]
    assert rows[0][1:] == ["8", "0.200", "25.00", "80.00"]
    assert rows[1][1:] == ["10", "0.050", "5.00", "20.00"]
