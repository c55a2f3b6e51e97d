"""The profile summariser (paper_2603_10634_amd.profile_summary) on small
hand-made rocprofv3 CSV files: the HBM byte counters are scaled by what they
read for the plain 1 GiB calibration copy, averaged per kernel and grid,
summed over the residue-product launches into the record the benchmark reads
(with the GEMM source's hash), and the kernel-trace table is written from the
statistics file."""
import csv
import json

import pytest

from paper_2603_10634_amd import profile_summary as ps

COUNTER_FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
NS = "void oz2::(anonymous namespace)::"


def _counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COUNTER_FIELDS)
        w.writeheader()
        for q, (name, grid, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": q + 1, "Grid_Size": grid, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_scales_by_the_copy_and_sums_the_products(tmp_path):
    sq = NS + "k_residue_gemm<0, false>(oz2::Problem, oz2::Group, int)"
    ka = NS + "k_residue_gemm<1, false>(oz2::Problem, oz2::Group, int)"
    crt = NS + "k_crt<4, 12, false>(oz2::Problem, oz2::Group)"
    copy = "__amd_rocclr_copyBuffer"
    # FETCH_SIZE reads half of the copy's 1 GiB (scale 2), WRITE_SIZE all of it
    _counters(tmp_path / "f_counter_collection.csv", "FETCH_SIZE",
              [(copy, 131072, 524288.0), (sq, 3145728, 1000.0), (sq, 3145728, 3000.0),
               (ka, 3145728, 5000.0), (crt, 67108864, 4000.0), (copy, 64, 0.5)])
    _counters(tmp_path / "w_counter_collection.csv", "WRITE_SIZE",
              [(copy, 131072, 1048576.0), (sq, 3145728, 1500.0), (ka, 3145728, 2500.0),
               (crt, 67108864, 6000.0)])
    md, js = tmp_path / "t.md", tmp_path / "t.json"
    ps.traffic(str(tmp_path), "f", "w", str(md), str(js), "cmd one ;; cmd two")
    rec = json.loads(js.read_text())
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # square launches averaged (2000 KiB), plus the Karatsuba one, in bytes
    assert rec["fetch_bytes_per_call"] == pytest.approx((2000.0 + 5000.0) * 1024 * 2)
    assert rec["write_bytes_per_call"] == pytest.approx((1500.0 + 2500.0) * 1024)
    assert rec["bytes_per_call"] == pytest.approx(rec["fetch_bytes_per_call"] +
                                                  rec["write_bytes_per_call"])
    assert rec["gemm_source_sha256"] == ps.gemm_source_sha()
    text = md.read_text()
    assert "    cmd one\n    cmd two\n" in text
    assert "| `k_crt<4, 12, false>` | 67108864 | 8.2 | 6.1 |" in text
    assert "| `__amd_rocclr_copyBuffer` | 64 |" not in text        # below 1 MB


def test_traffic_needs_the_calibration_copy(tmp_path):
    _counters(tmp_path / "f_counter_collection.csv", "FETCH_SIZE", [(NS + "k_x()", 1, 10.0)])
    _counters(tmp_path / "w_counter_collection.csv", "WRITE_SIZE", [(NS + "k_x()", 1, 10.0)])
    with pytest.raises(SystemExit):
        ps.traffic(str(tmp_path), "f", "w", str(tmp_path / "a.md"), str(tmp_path / "a.json"))


def test_trace_table(tmp_path):
    fields = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
              "StdDev"]
    with open(tmp_path / "tr_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerow({"Name": NS + "k_residue_gemm<1, false>(oz2::Problem, oz2::Group, int)",
                    "Calls": 15, "TotalDurationNs": 1, "AverageNs": 7238068.1,
                    "Percentage": 40.56, "MinNs": 7117853, "MaxNs": 7850728, "StdDev": 1})
    out = tmp_path / "trace.md"
    ps.trace(str(tmp_path), "tr", str(out), "the command")
    text = out.read_text()
    assert "    the command\n" in text
    assert "| `k_residue_gemm<1, false>` | 15 | 7.2381 | 7.1179 | 7.8507 | 40.56 |" in text
