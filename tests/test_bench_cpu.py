"""Host-side arithmetic of the benchmark's measurement record, on the CPU:
the nearest-rank percentile, the parsing of rocprofv3 counter output, the
search kernel's counter record assembled over both instantiations of the
pass and scaled by the plain-copy calibration, and the roofline record's
choice of the binding roof.  Records are written to a temporary directory,
never over the committed profiles."""
import csv
import json
import os

import pytest

import bench

K_RS = "vi::k_pass<false, false, false>"
K_GQ = "vi::k_pass<false, false, true>"
K_WIDE = "vi::k_pass_wide<64, false>"
COPY = bench.COPY_KERNEL


def test_nearest_rank_percentile():
    xs = list(range(1, 21))  # 20 timed steps
    assert bench.percentile(xs, 0.5) == 10
    assert bench.percentile(xs, 0.99) == 20  # ceil(0.99 * 20) = 20th smallest
    assert bench.percentile([5, 1, 4, 2, 3], 0.2) == 1
    assert bench.percentile([5, 1, 4, 2, 3], 0.6) == 3
    assert bench.percentile([7.5], 0.99) == 7.5


def test_summarize_counters_means_per_kernel_and_grid(tmp_path):
    d = tmp_path / "pmc"
    d.mkdir()
    fields = ["Kernel_Name", "Grid_Size", "Dispatch_Id", "Start_Timestamp", "End_Timestamp",
              "Counter_Name", "Counter_Value"]
    rows = [
        # two dispatches of one kernel at one grid, 10 us and 30 us
        {"Kernel_Name": K_RS + "(vi::DevLevel, vi::PassArgs)", "Grid_Size": 512, "Dispatch_Id": 1,
         "Start_Timestamp": 1000, "End_Timestamp": 11000, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 100.0},
        {"Kernel_Name": K_RS + "(vi::DevLevel, vi::PassArgs)", "Grid_Size": 512, "Dispatch_Id": 2,
         "Start_Timestamp": 20000, "End_Timestamp": 50000, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 300.0},
        # another grid of the same kernel
        {"Kernel_Name": "void " + K_RS + "(vi::DevLevel, vi::PassArgs)", "Grid_Size": 256,
         "Dispatch_Id": 3, "Start_Timestamp": 0, "End_Timestamp": 4000,
         "Counter_Name": "FETCH_SIZE", "Counter_Value": 8.0},
    ]
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)
    out = {(r["kernel"], r["grid"]): r for r in bench.summarize_counters(str(tmp_path))}
    a = out[(K_RS, 512)]
    assert a["dispatches"] == 2
    assert a["mean_us"] == pytest.approx(20.0)
    assert a["counters"]["FETCH_SIZE"] == pytest.approx(200.0)
    b = out[(K_RS, 256)]
    assert b["dispatches"] == 1 and b["mean_us"] == pytest.approx(4.0)


def _summary(path, rows):
    with open(path, "w") as f:
        json.dump(rows, f)
    return str(path)


def _pass_rows(counter, values):
    # (kernel, grid, dispatches, mean_us, counter value)
    return [{"kernel": k, "grid": g, "dispatches": n, "mean_us": us, "counters": {counter: v}}
            for k, g, n, us, v in values]


def test_assemble_counters_over_both_instantiations(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "counters_json",
                        lambda w: str(tmp_path / f"k_pass_{w}_counters.json"))
    shape = [(K_RS, 2048, 1, 100.0), (K_GQ, 2048, 3, 20.0), (K_WIDE, 512, 5, 9.0)]
    fetch = _summary(tmp_path / "f.json", _pass_rows(
        "FETCH_SIZE", [s + (v,) for s, v in zip(shape, (1000.0, 200.0, 7.0))]))
    write = _summary(tmp_path / "w.json", _pass_rows(
        "WRITE_SIZE", [s + (v,) for s, v in zip(shape, (40.0, 8.0, 1.0))]))
    sq_vals = {c: 0.0 for c in bench.SQ_COUNTERS.split()}
    sq_rows = []
    for (k, g, n, us), valu in zip(shape, (6.0e6, 1.0e6, 5.0)):
        c = dict(sq_vals, SQ_INSTS_VALU=valu, SQ_INSTS_LDS=10.0, SQ_LDS_BANK_CONFLICT=5.0)
        sq_rows.append({"kernel": k, "grid": g, "dispatches": n, "mean_us": us, "counters": c})
    sq = _summary(tmp_path / "s.json", sq_rows)
    # a plain 1 GiB copy: FETCH_SIZE reads half the bytes (factor 2), WRITE_SIZE all (factor 1)
    cfetch = _summary(tmp_path / "cf.json", _pass_rows(
        "FETCH_SIZE", [(COPY, 1, 2, 400.0, bench.COPY_BYTES / 1024 / 2)]))
    cwrite = _summary(tmp_path / "cw.json", _pass_rows(
        "WRITE_SIZE", [(COPY, 1, 2, 400.0, bench.COPY_BYTES / 1024)]))
    rec = bench.assemble_counters(fetch, write, sq, cfetch, cwrite, "unit")
    # dispatch-weighted means over the two instantiations; the wide kernel is not included
    fk = (1 * 1000.0 + 3 * 200.0) / 4
    wk = (1 * 40.0 + 3 * 8.0) / 4
    assert rec["dispatches"] == 4
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(1024.0 * (2.0 * fk + 1.0 * wk))
    assert rec["mean_launch_us"] == pytest.approx((1 * 100.0 + 3 * 20.0) / 4)
    valu = (1 * 6.0e6 + 3 * 1.0e6) / 4
    assert rec["valu_busy"] == pytest.approx(valu / (256 * 40.0 * 2400.0))
    assert {(r["kernel"], r["grid"]) for r in rec["per_grid"]} == {(K_RS, 2048), (K_GQ, 2048)}
    assert rec["source_sha256"] == bench.kernel_source_hash()
    with open(tmp_path / "k_pass_unit_counters.json") as f:
        assert json.load(f)["hbm_bytes_per_launch"] == rec["hbm_bytes_per_launch"]


def _counter_record(path, valu_busy, hbm_bytes, mean_us, source):
    rec = {"source_sha256": source, "hbm_bytes_per_launch": hbm_bytes,
           "mean_launch_us": mean_us, "valu_busy": valu_busy,
           # 2 GiB moved in 400 us: the copy rate
           "copy_calibration": {"bytes": bench.COPY_BYTES, "mean_us": 400.0}}
    with open(path, "w") as f:
        json.dump(rec, f)


@pytest.mark.parametrize("valu_busy,expect", [(0.2, "hbm"), (0.9, "alu")])
def test_roofline_takes_the_roof_nearer_saturation(tmp_path, monkeypatch, valu_busy, expect):
    path = str(tmp_path / "rec.json")
    monkeypatch.setattr(bench, "counters_json", lambda w: path)
    copy_gbs = 2.0 * bench.COPY_BYTES / 400e-6 / 1e9
    # measured traffic at half the copy rate
    mean_us = 100.0
    hbm_bytes = 0.5 * copy_gbs * 1e9 * mean_us * 1e-6
    _counter_record(path, valu_busy, hbm_bytes, mean_us, bench.kernel_source_hash())
    evals, units, ms, launches = 4.0e6, 3.0e7, 20.0, 200
    r = bench.roofline_of("unit", evals, units, ms, launches, nominal_pass=1.0e9)
    avg_s = ms / launches * 1e-3
    gbs = (bench.BYTES_PER_EVAL * evals / launches
           + bench.BYTES_PER_TARGET_PASS * units / launches) / avg_s / 1e9
    tops = bench.OPS_PER_EVAL * evals / launches / avg_s / 1e12
    assert r["bound"] == expect
    if expect == "hbm":
        assert r["achieved"] == pytest.approx(gbs, rel=1e-3)
        assert r["peak"] == bench.HBM_PEAK_GBS and r["unit"] == "GB/s"
    else:
        assert r["achieved"] == pytest.approx(tops, rel=1e-3)
        assert r["unit"] == "TOP/s"
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)  # 4 decimals
    assert r["traffic"] == round(hbm_bytes)
    assert r["counters"]["hbm_frac_of_copy"] == pytest.approx(0.5, rel=1e-3)


def test_roofline_ignores_counters_of_another_source(tmp_path, monkeypatch):
    path = str(tmp_path / "rec.json")
    monkeypatch.setattr(bench, "counters_json", lambda w: path)
    _counter_record(path, 0.9, 1.0e8, 100.0, "0" * 64)
    r = bench.roofline_of("unit", 4.0e6, 3.0e7, 20.0, 200, nominal_pass=1.0e9)
    assert r["counters"] is None and r["traffic"] is None and r["bound"] == "hbm"
