"""The rocprofv3 summaries behind the committed profiles
(paper_1805_05821_amd/rocprof_summary.py), on small synthetic trace and
counter files whose answers are known by construction."""

import csv
import json
import os

import pytest

from paper_1805_05821_amd import rocprof_summary as RS


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _trace(tmp_path, durations_ms, name="void foa::k_x<float, 8>(foa::Args)", other=2):
    """Kernel trace: the given durations of one kernel in time order, with
    `other` dispatches of a second kernel interleaved (ns timestamps)."""
    rows, t = [], 1_000_000
    for i, d in enumerate(durations_ms):
        rows.append([name, t, t + int(round(d * 1e6))])
        t += int(round(d * 1e6)) + 5_000
        if i < other:
            rows.append(["void foa::k_y(foa::Args)", t, t + 1_000_000])
            t += 1_005_000
    d = tmp_path / "trace"
    _write_csv(str(d / "run" / "t_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    return str(d)


def test_window_picks_dispatches_in_time_order(tmp_path):
    d = _trace(tmp_path, [1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    out = RS.window(d, "void foa::k_x", 2, 3)
    # dispatches 2..4 of 6: 3 + 4 + 5 ms
    assert "dispatches 2..4 of 6" in out
    assert "total 12.00 ms, average 4.0000 ms" in out


def test_window_counts_short_dispatches_apart(tmp_path):
    # a gated kernel: half of its dispatches return at once (4 us)
    d = _trace(tmp_path, [0.004, 2.0, 0.004, 4.0, 0.004, 6.0], other=0)
    out = RS.window(d, "void foa::k_x", 0, 6, 20)
    assert "3 ran, total 12.00 ms, average 4.0000 ms" in out
    assert "3 under 20 us (returned at once), total 0.01 ms" in out


def _counters(path, per_dispatch):
    """counter_collection.csv: per_dispatch = [(kernel, counter, [values per
    dispatch, each split over two instances as rocprofv3 reports them])]."""
    rows, disp = [], 0
    for kernel, counter, values in per_dispatch:
        for v in values:
            disp += 1
            rows.append([disp, kernel, counter, v / 2.0])
            rows.append([disp, kernel, counter, v / 2.0])
    _write_csv(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_counter_per_dispatch_sums_instances(tmp_path):
    p = str(tmp_path / "c" / "x_counter_collection.csv")
    _counters(p, [("k_a", "FETCH_SIZE", [10.0, 30.0]), ("k_b", "FETCH_SIZE", [5.0])])
    per = RS.counter_per_dispatch(str(tmp_path / "c"), "FETCH_SIZE")
    assert per["k_a"] == (40.0, 2) and per["k_b"] == (5.0, 1)


def test_kernel_traffic_scales_by_the_copy(tmp_path):
    copy_bytes = 4 << 30
    # the copy reads copy_bytes and FETCH_SIZE reports 2^21 units: 2048 bytes per unit;
    # it writes copy_bytes and WRITE_SIZE reports 2^22 units: 1024 bytes per unit
    _counters(str(tmp_path / "fc" / "c_counter_collection.csv"), [("__amd_rocclr_copyBuffer", "FETCH_SIZE", [2.0 ** 21])])
    _counters(str(tmp_path / "wc" / "c_counter_collection.csv"), [("__amd_rocclr_copyBuffer", "WRITE_SIZE", [2.0 ** 22])])
    _counters(str(tmp_path / "f" / "k_counter_collection.csv"),
              [("void foa::k_ls_pass<float>", "FETCH_SIZE", [1000.0, 3000.0]), ("void foa::other", "FETCH_SIZE", [7.0])])
    _counters(str(tmp_path / "w" / "k_counter_collection.csv"), [("void foa::k_ls_pass<float>", "WRITE_SIZE", [100.0, 100.0])])
    log = tmp_path / "bench.log"
    alg = 2000.0 * 2048 + 100.0 * 1024
    log.write_text("noise\n" + json.dumps({"sweep_alg_bytes_per_launch": alg}) + "\n")
    r = RS.kernel_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "fc"), str(tmp_path / "wc"),
                          copy_bytes, "void foa::k_ls_pass<", str(log), "sweep_alg_bytes_per_launch")
    assert r["dispatches"] == [2, 2]
    assert r["fetch_scale"] == pytest.approx(2048.0) and r["write_scale"] == pytest.approx(1024.0)
    assert r["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 2048)
    assert r["write_bytes_per_launch"] == pytest.approx(100.0 * 1024)
    assert r["traffic_over_alg"] == pytest.approx(1.0)


def test_counter_window_picks_dispatches_in_order_and_scales(tmp_path):
    copy_bytes = 4 << 30
    _counters(str(tmp_path / "fc" / "c_counter_collection.csv"), [("__amd_rocclr_copyBuffer", "FETCH_SIZE", [2.0 ** 21])])
    _counters(str(tmp_path / "wc" / "c_counter_collection.csv"), [("__amd_rocclr_copyBuffer", "WRITE_SIZE", [2.0 ** 22])])
    # four dispatches of the kernel (two runs of two), another kernel in between
    _counters(str(tmp_path / "f" / "k_counter_collection.csv"),
              [("void foa::k_bpass<float, 1>", "FETCH_SIZE", [10.0, 20.0]), ("void foa::other", "FETCH_SIZE", [7.0]),
               ("void foa::k_bpass<float, 1>", "FETCH_SIZE", [100.0, 300.0])])
    _counters(str(tmp_path / "w" / "k_counter_collection.csv"),
              [("void foa::k_bpass<float, 1>", "WRITE_SIZE", [1.0, 1.0, 4.0, 6.0])])
    r = RS.counter_window(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "fc"), str(tmp_path / "wc"),
                          copy_bytes, "void foa::k_bpass<float", 2, 2)
    assert r["dispatches"] == [2, 2] and r["of"] == [4, 4]
    assert r["fetch_bytes_per_launch"] == pytest.approx(200.0 * 2048)
    assert r["write_bytes_per_launch"] == pytest.approx(5.0 * 1024)
