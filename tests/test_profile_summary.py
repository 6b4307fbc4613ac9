"""The rocprofv3 summary tool on synthetic CSV files (no GPU): kernel-name
shortening, the per-dispatch readers, and the tail summary's arithmetic
(average duration, counter bytes scaled per launch and per state, the
rate by the algorithmic bytes)."""
import argparse
import csv
import os

import numpy as np

from paper_2603_07341_amd import profile_summary as ps

MID = "k_cheb_term<double, 1, 1, true>"
LONG = ("void paces::(anonymous namespace)::k_cheb_term<double, 1, 1, true>"
        "(paces::DevModel, int, int)")


def write_csv(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_short_name():
    assert ps.short_name(LONG) == MID
    assert ps.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_tail_summary_arithmetic(tmp_path):
    tr, fe, wr = (tmp_path / d for d in ("trace", "fetch", "write"))
    for d in (tr, fe, wr):
        os.makedirs(d)
    # six launches: two other kernels and four of the middle term
    # (durations 1, 2, 3, 4 ms); the last two are the tail
    names = ["k_bounds<4>", LONG, LONG, "k_pop_norm<double>", LONG, LONG]
    dur = [5, 1_000_000, 2_000_000, 7, 3_000_000, 4_000_000]
    write_csv(tr / "run_kernel_trace.csv",
              ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
              [{"Dispatch_Id": i, "Kernel_Name": n, "Start_Timestamp": 100 * i,
                "End_Timestamp": 100 * i + d}
               for i, (n, d) in enumerate(zip(names, dur))])
    # counters in KiB per dispatch, split over two rows (summed per dispatch)
    rows_f, rows_w = [], []
    for i, n in enumerate(names):
        for part in (0, 1):
            rows_f.append({"Dispatch_Id": i, "Kernel_Name": n,
                           "Counter_Name": "FETCH_SIZE", "Counter_Value": 500 * (i + 1)})
            rows_w.append({"Dispatch_Id": i, "Kernel_Name": n,
                           "Counter_Name": "WRITE_SIZE", "Counter_Value": 100 * (i + 1)})
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    write_csv(fe / "run_counter_collection.csv", fields, rows_f)
    write_csv(wr / "run_counter_collection.csv", fields, rows_w)
    rec = np.zeros((5, 12))
    rec[:, 7] = [10, 20, 30, 1000, 3000]  # states of the steps
    np.save(tmp_path / "rec.npy", rec)
    out = tmp_path / "tail.txt"
    args = argparse.Namespace(
        trace=str(tr), fetch=str(fe), write=str(wr),
        records=str(tmp_path / "rec.npy"), kernel=MID, last=2, steps=2,
        alg_bytes=108, fetch_scale=2.0, write_scale=1.0,
        command="python3 bench.py", title="synthetic", out=str(out))
    text = ps.summarize_tail(args)
    vals = dict(l.split(": ", 1) for l in text.splitlines()
                if ": " in l and not l.startswith("#"))
    # the last two middle launches: dispatches 4 and 5
    assert vals["launches_used"].startswith("2 (the last of 4)")
    assert float(vals["avg_us"]) == 3500.0
    fetch = (2 * 500 * 5 + 2 * 500 * 6) / 2 * 1024 * 2.0
    write = (2 * 100 * 5 + 2 * 100 * 6) / 2 * 1024 * 1.0
    assert float(vals["counted_fetch_bytes_per_launch"]) == fetch
    assert float(vals["counted_write_bytes_per_launch"]) == write
    states = 2000.0  # mean of the last two records
    assert abs(float(vals["counted_bytes_per_state"]) - (fetch + write) / states) < 0.06
    frac = 108 * states / 3500e-6 / 8e12
    assert abs(float(vals["algorithmic_frac_of_8tbs"]) - frac) < 5e-4
    assert out.read_text() == text


def test_stage_bandwidth_reports_in_place_transfer_with_the_expansion():
    """bench.stage_bandwidth: algorithmic bytes per stage from the records
    over event time; with in-place steps the transfer has no rate of its
    own and is reported with the expansion."""
    import bench

    class M:
        W, D = 2, 4
    A = 16
    srec = np.zeros((2, 12))
    srec[:, 7] = [1000.0, 1100.0]   # |S|
    srec[:, 8] = [400.0, 420.0]     # |M|
    srec[:, 9] = [10.0, 10.0]       # K
    ms = {"select": 1.0, "expand": 2.0, "transfer": 0.5, "build": 1.0,
          "propagate": 10.0, "observe": 1.0}
    out = bench.stage_bandwidth(M, A, {"ms": ms}, srec, 900.0, 2, 5000.0,
                                None, in_place=True)
    assert out["transfer"]["effective"] is None
    prop = (1000 * 10 + 1100 * 10) * (4 * A + 4 * M.D + 8)
    assert abs(out["propagate"]["bytes_per_step"] - prop / 2) < 1e-6
    assert abs(out["propagate"]["effective"] - prop / 10e-3 / 1e9) < 1e-9
    both = out["expand+transfer+build"]
    assert abs(both["ms_per_step"] - (2.0 + 1.0 + 0.5) / 2) < 1e-12
    plain = bench.stage_bandwidth(M, A, {"ms": ms}, srec, 900.0, 2, 5000.0,
                                  None, in_place=False)
    assert plain["transfer"]["effective"] > 0
