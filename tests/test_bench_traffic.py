"""Host logic of bench.py's walk traffic figures: rocprofv3 counter rows
(FETCH_SIZE and WRITE_SIZE, KiB per dispatch) scaled by a copy of known
size, per walk kernel instance; no GPU."""
import argparse
import csv
import os

import pytest

import bench

COPY_MIB = 512


def _rows(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})
    return d


def _copy_dirs(tmp):
    # the copy reads FETCH_SIZE at half its bytes and WRITE_SIZE at its bytes
    kib = COPY_MIB * 1024
    cf = _rows(os.path.join(tmp, "cf"), "FETCH_SIZE", [("__amd_rocclr_copyBuffer", kib / 2)] * 2)
    cw = _rows(os.path.join(tmp, "cw"), "WRITE_SIZE", [("__amd_rocclr_copyBuffer", kib)] * 2)
    return cf, cw


def _args(precision, workload, theta, waves, group):
    return argparse.Namespace(
        precision=precision, workload=workload, theta=theta, leaf_size=1, group_size=group,
        split_images=0, walk_waves=waves, calibrate_copy=COPY_MIB,
        write_traffic=None)


@pytest.mark.parametrize("precision,waves,timed,other", [
    ("fp64", 1, "k_walk64<true, false, 1, true>", "k_walk64<true, true, 1, false>"),
    ("fp32", 1, "k_walk32<true, false>", "k_walk32<true, true>"),
    ("fp32", 4, "k_walk32m<true, false, 4>", "k_walk32m<true, true, 4>"),
])
def test_walk_traffic_scales_the_timed_launches(tmp_path, precision, waves, timed, other):
    tmp = str(tmp_path)
    cf, cw = _copy_dirs(tmp)
    # three timed launches (median 2000 KiB fetched, 500 written) and a stats
    # launch of the same kernel, which must not count
    wf = _rows(os.path.join(tmp, "wf"), "FETCH_SIZE",
               [(timed, 1000.0), (timed, 2000.0), (timed, 9000.0), (other, 1e9)])
    ww = _rows(os.path.join(tmp, "ww"), "WRITE_SIZE",
               [(timed, 500.0), (timed, 400.0), (timed, 600.0), (other, 1e9)])
    a = _args(precision, "sheet50k", 0.3, waves, 64)
    a.write_traffic = [cf, cw, wf, ww]
    meta = bench.write_traffic(a, out_dir=tmp)
    assert meta["dispatches"] == 3
    assert meta["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert meta["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    assert meta["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert meta["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert meta["bytes_per_launch"] == pytest.approx((4000.0 + 500.0) * 1024)
    assert meta["source_sha256"] == bench.walk_source_sha(precision)
    if precision == "fp64":  # the FP64 walk has no groups or waves per item
        assert meta["knobs"]["group_size"] is None and meta["knobs"]["walk_waves"] is None
    else:
        assert meta["knobs"]["group_size"] == 64 and meta["knobs"]["walk_waves"] == waves


def test_walk_traffic_keeps_one_entry_per_operating_point(tmp_path):
    tmp = str(tmp_path)
    cf, cw = _copy_dirs(tmp)
    name = "k_walk64<true, false, 2, true>"
    wf = _rows(os.path.join(tmp, "wf"), "FETCH_SIZE", [(name, 10.0)])
    ww = _rows(os.path.join(tmp, "ww"), "WRITE_SIZE", [(name, 20.0)])
    for theta in (0.26, 0.3, 0.26):
        a = _args("fp64", "sheet50k", theta, 1, 64)
        a.write_traffic = [cf, cw, wf, ww]
        bench.write_traffic(a, out_dir=tmp)
    entries = bench.traffic_entries(os.path.join(tmp, "walk_fp64_sheet50k_traffic.json"))
    assert sorted(e["knobs"]["theta"] for e in entries) == [0.26, 0.3]


def test_walk_traffic_needs_rows_of_the_kernel(tmp_path):
    tmp = str(tmp_path)
    cf, cw = _copy_dirs(tmp)
    wf = _rows(os.path.join(tmp, "wf"), "FETCH_SIZE", [("k_walk32<true, false>", 10.0)])
    ww = _rows(os.path.join(tmp, "ww"), "WRITE_SIZE", [("k_walk32<true, false>", 10.0)])
    a = _args("fp64", "sheet50k", 0.26, 1, 64)
    a.write_traffic = [cf, cw, wf, ww]
    with pytest.raises(SystemExit):
        bench.write_traffic(a, out_dir=tmp)
