"""Host logic of the rocprofv3 summaries (paper_2602_12314_amd.profiling) on
small synthetic CSV files of the profiler's column layout."""
import csv
import json
import os

from paper_2602_12314_amd import profiling

TRACE_COLS = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"]
PMC_COLS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(path, cols, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(cols)
        w.writerows(rows)


def _trace(tmp_path):
    # two steps: projection, rows, then dV beside the compositing backward
    rows = []
    for t0 in (0, 10_000_000, 20_000_000):
        rows += [
            ["void lam::k_preprocess(lam::CamSet, int)", 1000, 1, 1, t0, t0 + 40_000],
            ["void lam::k_dec_rows<lam::TBF16, 4>(lam::RowsArgs)", 64, 1, 1, t0 + 50_000, t0 + 4_050_000],
            ["void lam::k_dec_dv<lam::TBF16, 32, 2>(float const*)", 128, 1, 1, t0 + 4_060_000, t0 + 6_060_000],
            ["void lam::k_raster_bwd<32, false, false>(lam::CamSet)", 256, 1, 1, t0 + 4_070_000, t0 + 5_070_000],
        ]
    _write(str(tmp_path / "tr" / "run_kernel_trace.csv"), TRACE_COLS, rows)
    return str(tmp_path / "tr")


def test_stats_by_grid_groups_kernel_and_grid(tmp_path):
    d = _trace(tmp_path)
    rows = profiling.kernel_stats_by_grid(d)
    by = {(k, g): (calls, tot, avg) for k, g, calls, tot, avg in rows}
    assert by[("k_dec_rows<TBF16, 4>", 64)] == (3, 12_000.0, 4_000.0)
    assert by[("k_raster_bwd<32, false, false>", 256)][2] == 1_000.0
    assert rows[0][0] == "k_dec_rows<TBF16, 4>"  # largest total first


def test_timeline_prints_one_step_in_start_order(tmp_path, capsys):
    d = _trace(tmp_path)
    assert profiling.main(["timeline", d, "--step", "1"]) == 0
    out = capsys.readouterr().out.splitlines()
    body = [ln for ln in out if ln.startswith("| ") and not ln.startswith("| start")]
    assert [ln.split(" | ")[3] for ln in body] == [
        "k_preprocess", "k_dec_rows<TBF16, 4>", "k_dec_dv<TBF16, 32, 2>", "k_raster_bwd<32, false, false>"]
    # relative to the step's first launch, in microseconds
    assert body[2].startswith("| 4060.00 | 6060.00 | 2000.00 |")
    assert out[-1] == "next step's projection starts at 10000.00 us"


def test_traffic_scales_by_copy_calibration_and_records_json(tmp_path):
    gib = 1 << 30
    # the copy kernel's counters read half the bytes it fetched and all it wrote
    _write(str(tmp_path / "cf" / "run_counter_collection.csv"), PMC_COLS,
           [["__amd_rocclr_copyBuffer", 64, "FETCH_SIZE", gib / 2048.0]])
    _write(str(tmp_path / "cw" / "run_counter_collection.csv"), PMC_COLS,
           [["__amd_rocclr_copyBuffer", 64, "WRITE_SIZE", gib / 1024.0]])
    # two grids of the rows kernel; --largest-grid keeps the larger one only
    _write(str(tmp_path / "f" / "run_counter_collection.csv"), PMC_COLS,
           [["void lam::k_dec_rows<lam::TBF16, 4>(x)", 100, "FETCH_SIZE", 10.0],
            ["void lam::k_dec_rows<lam::TBF16, 4>(x)", 200, "FETCH_SIZE", 1000.0],
            ["void lam::k_dec_rows<lam::TBF16, 4>(x)", 200, "FETCH_SIZE", 3000.0]])
    _write(str(tmp_path / "w" / "run_counter_collection.csv"), PMC_COLS,
           [["void lam::k_dec_rows<lam::TBF16, 4>(x)", 200, "WRITE_SIZE", 500.0]])
    js = str(tmp_path / "traffic.json")
    args = ["traffic", "--workload", "wl", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"),
            "--copy-fetch", str(tmp_path / "cf"), "--copy-write", str(tmp_path / "cw"),
            "--copy-bytes", str(gib), "--largest-grid", "--json", js, "--only", "decode_rows",
            "--options", '{"precision": "fp8"}']
    assert profiling.main(args) == 0
    ent = json.load(open(js))["wl"]["decode_rows"]
    assert ent["fetch_factor"] == 2.0 and ent["write_factor"] == 1.0
    assert ent["fetch_kib"] == 2000.0 and ent["write_kib"] == 500.0
    assert ent["bytes_per_launch"] == 2000.0 * 1024 * 2 + 500.0 * 1024
    assert ent["options"] == {"precision": "fp8"}
    assert ent["source_hash"] == profiling.source_hash(profiling.STAGES["decode_rows"][1])
