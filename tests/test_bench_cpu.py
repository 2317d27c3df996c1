"""bench.py's host logic on the CPU: the one-GPU guard, the reduction of
rocprofv3 counter files to per-launch HBM traffic (copy-calibrated) and to the
VALU issue rate, and the tuning-to-arguments conversion."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path):
    # the copy reads and writes 1 GiB; its FETCH_SIZE reads half of that (scale 2), WRITE_SIZE all of it
    gib_kib = float(1 << 20)
    _write(tmp_path / "copy_fetch", "FETCH_SIZE", [("at::native::neg_kernel", gib_kib / 2)] * 3)
    _write(tmp_path / "copy_write", "WRITE_SIZE", [("at::native::neg_kernel", gib_kib)] * 3)
    dens = "void clue::k_density<true, 2, 0>(clue::DescArg<true>, clue::Geom, clue::Arena)"
    lab = "void clue::k_label<true>(clue::DescArg<true>, clue::Geom, clue::Arena)"
    _write(tmp_path / "fetch", "FETCH_SIZE", [(dens, 1000.0), (dens, 1200.0), (lab, 50.0),
                                             ("void clue::k_density<false, 2, 0>(x)", 9e9)])
    _write(tmp_path / "write", "WRITE_SIZE", [(dens, 300.0), (dens, 300.0), (lab, 25.0)])
    out = tmp_path / "traffic.json"
    bench.traffic_summary(str(tmp_path), "density", 32, out_path=str(out))
    t = json.loads(out.read_text())
    assert t["scale_fetch"] == pytest.approx(2.0) and t["scale_write"] == pytest.approx(1.0)
    # mean over the batched density dispatches only (the plain one is excluded)
    assert t["fetch_kib_per_dispatch"] == pytest.approx(1100.0)
    assert t["hbm_bytes_per_launch"] == pytest.approx(1100.0 * 1024 * 2 + 300.0 * 1024)
    assert t["hits_per_launch"] == 32 * 10 ** 6
    assert t["per_stage_hbm_bytes_per_launch"]["labels"] == pytest.approx(50.0 * 1024 * 2 + 25.0 * 1024)
    assert "grid_hist" not in t["per_stage_hbm_bytes_per_launch"]
    assert t["kernel_source_sha"] == bench.kernel_source_sha()


def test_issue_summary_divides_valu_by_cu_cycles(tmp_path):
    dens = "void clue::k_density<true, 2, 0>(clue::DescArg<true>, clue::Geom, clue::Arena)"
    _write(tmp_path / "sq", "SQ_INSTS_VALU", [(dens, 6.0e8), (dens, 6.2e8),
                                             ("void clue::k_density<false, 2, 0>(x)", 1.0)])
    os.makedirs(tmp_path / "ktrace")
    with open(tmp_path / "ktrace" / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": dens, "Calls": 10, "AverageNs": 1.0e6})
    out = tmp_path / "issue.json"
    bench.issue_summary(str(tmp_path), "density", 32, out_path=str(out))
    t = json.loads(out.read_text())
    assert t["sq_insts_valu_per_launch"] == pytest.approx(6.1e8)
    # 256 CUs x 1 ms x 2.4 GHz = 6.144e8 CU-cycles
    assert t["valu_insts_per_cu_cycle"] == pytest.approx(6.1e8 / 6.144e8)
    assert t["kernel_source_sha"] == bench.kernel_source_sha() and t["hits_per_launch"] == 32 * 10 ** 6


def test_overlap_summary_measures_time_with_two_streams_busy(tmp_path):
    # stream 1 runs [0, 10) and [20, 30), stream 2 runs [5, 25): both are busy
    # in [5, 10) and [20, 25), some stream in [0, 30); non-CLUE kernels are ignored
    rows = [("clue::k_density", 1, 0, 10), ("clue::k_label", 1, 20, 30), ("clue::k_hist", 2, 5, 25),
            ("at::native::neg_kernel", 3, 0, 30)]
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Stream_Id", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, st, t0, t1 in rows:
            w.writerow({"Kernel_Name": name, "Stream_Id": st, "Start_Timestamp": t0 * 10 ** 6,
                        "End_Timestamp": t1 * 10 ** 6})
    o = bench.overlap_summary(str(tmp_path))
    assert o["kernels_per_stream"] == {"1": 2, "2": 1}
    assert o["span_ms"] == pytest.approx(30.0) and o["busy_ms"] == pytest.approx(30.0)
    assert o["two_or_more_in_flight_ms"] == pytest.approx(10.0)
    assert o["frac_of_busy_two_or_more"] == pytest.approx(1 / 3)


def test_linear_fit_recovers_a_line():
    xs = [1e5 * k for k in range(1, 11)]
    f = bench.linear_fit(xs, [0.2 + 0.13e-6 * x for x in xs])
    assert f["slope_ms_per_Mhit"] == pytest.approx(0.13) and f["intercept_ms"] == pytest.approx(0.2)
    assert f["r2"] == pytest.approx(1.0)


def test_code_sha_ignores_comments_and_spacing_only():
    a = "int f(int x) {\n  return x + 1;  // one more\n}\n"
    b = "/* header */ int f(int x) { return x + 1; }"
    c = "int f(int x) { return x + 2; }"
    assert bench.code_sha([a]) == bench.code_sha([b]) != bench.code_sha([c])


def test_tuning_kwargs():
    t = {"block": (10, 8), "tile_size": 4.0, "lds_cap": 768, "plain_lds_cap": 960, "ms": 4.8, "density_quads": 1}
    kw = bench.tuning_kwargs(t)
    assert kw == {"block_x": 10, "block_y": 8, "tile_size": 4.0, "lds_cap": 768, "plain_lds_cap": 960,
                  "density_quads": 1}
