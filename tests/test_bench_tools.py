"""Host logic of bench.py's profile tooling: the per-kernel counter summary
built from rocprofv3 csv output (no GPU; small csv files written here)."""
import csv
import os

import bench

COUNTER_FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
TRACE_FIELDS = ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def write_csv(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_counters(tmp_path):
    k1 = "void lsefit::k_moments<3, 0, float, 2>(lsefit::FitDesc, lsefit::Work)"
    k2 = "lsefit::k_finish_single<3>(lsefit::FitDesc)"
    other = "void at::native::elementwise_kernel<16>(int)"
    counters = []
    for did, (name, a, b) in enumerate([(k1, 10.0, 100.0), (k1, 30.0, 300.0), (k2, 4.0, 8.0), (other, 1e9, 1e9)]):
        counters.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": a})
        counters.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": "SQ_BUSY_CYCLES", "Counter_Value": b})
    trace = [{"Dispatch_Id": 0, "Kernel_Name": k1, "Start_Timestamp": 1000, "End_Timestamp": 121000},
             {"Dispatch_Id": 1, "Kernel_Name": k1, "Start_Timestamp": 200000, "End_Timestamp": 318000},
             {"Dispatch_Id": 2, "Kernel_Name": k2, "Start_Timestamp": 400000, "End_Timestamp": 408000},
             {"Dispatch_Id": 3, "Kernel_Name": other, "Start_Timestamp": 500000, "End_Timestamp": 900000}]
    sub = tmp_path / "pass"
    sub.mkdir()
    write_csv(sub / "run_counter_collection.csv", COUNTER_FIELDS, counters)
    write_csv(sub / "run_kernel_trace.csv", TRACE_FIELDS, trace)
    out = tmp_path / "summary.txt"
    bench.summarize_counters(str(tmp_path), "title", "the command", out_path=str(out))
    text = out.read_text().splitlines()
    assert text[0] == "# rocprofv3 counter summary: title"
    assert "#   the command" in text
    assert f"kernel_hash {bench.kernel_hash()}" in text
    body = [ln for ln in text if not ln.startswith("#") and not ln.startswith("kernel_hash")]
    # library kernels only, the longest in total first; averages per dispatch
    assert body[0] == "void lsefit::k_moments<3, 0, float, 2>  dispatches 2  avg 119.00 us"
    vals = {ln.split()[0]: ln.split()[1] for ln in body[1:3]}
    assert vals == {"SQ_BUSY_CYCLES": "200.0", "SQ_INSTS_VALU": "20.0"}
    assert body[3] == "lsefit::k_finish_single<3>  dispatches 1  avg 8.00 us"
    assert not any("elementwise" in ln for ln in text)
    assert os.path.getsize(out) < 4096


STATS_FIELDS = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]


def test_summarize_trace_timed_region(tmp_path, monkeypatch):
    """The trace summary averages the dispatches of the timed region (by launch
    order, skipping the warm-up ones) and bench.py reads that average back only
    while the kernel sources hash the same."""
    k1 = "void lsefit::k_moments<3, 0, float, 2>(lsefit::FitDesc, lsefit::Work)"
    k2 = "lsefit::k_finish_single<3>(lsefit::FitDesc)"
    trace, t = [], 0
    durs = [200, 150, 100, 110, 120, 900]          # 2 warm-up, 3 timed, 1 later (us)
    for i, d in enumerate(durs):
        trace.append({"Dispatch_Id": 2 * i, "Kernel_Name": k1, "Start_Timestamp": t, "End_Timestamp": t + d * 1000})
        t += d * 1000
        trace.append({"Dispatch_Id": 2 * i + 1, "Kernel_Name": k2, "Start_Timestamp": t, "End_Timestamp": t + 7000})
        t += 7000
    # rows out of launch order in the file: the summary sorts by start time
    trace = trace[::-1]
    stats = [{"Name": k1, "Calls": 6, "TotalDurationNs": 1580000, "AverageNs": 263333.3, "Percentage": 90,
              "MinNs": 100000, "MaxNs": 900000, "StdDev": 0},
             {"Name": k2, "Calls": 6, "TotalDurationNs": 42000, "AverageNs": 7000, "Percentage": 10,
              "MinNs": 7000, "MaxNs": 7000, "StdDev": 0}]
    sub = tmp_path / "run"
    sub.mkdir()
    write_csv(sub / "run_kernel_trace.csv", TRACE_FIELDS, trace)
    write_csv(sub / "run_kernel_stats.csv", STATS_FIELDS, stats)
    out = tmp_path / "trace.txt"
    bench.summarize_trace(str(tmp_path), "title", "the command", out_path=str(out),
                          timed=("k_moments<3, 0, float, 2>", "2", "3"))
    text = out.read_text().splitlines()
    timed = [ln for ln in text if ln.startswith("timed_region")]
    assert timed == ["timed_region k_moments<3, 0, float, 2> dispatches 2..4 of 6  "
                     "avg 110.00 us  min 100.00 us  max 120.00 us"]
    monkeypatch.setattr(bench, "TRACE_FILE", str(out))
    assert abs(bench.profile_timed_avg_ms() - 0.110) < 1e-12
    # another source hash: the stored figure no longer describes these kernels
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0000000000000000")
    assert bench.profile_timed_avg_ms() is None
