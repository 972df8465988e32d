"""Host: the rocprofv3 summary helpers (counter CSV -> traffic per launch; stats table)."""
import csv
import json

from paper_1601_04641_amd import profiling

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]

X128 = "void gpk::k_sweep_lines<double, 16, 8, true, 2, false, 8>(gpk::VecOf<double>::T*, long)"
Y128 = "void gpk::k_sweep_lines<double, 16, 4, true, 0, false, 16>(gpk::VecOf<double>::T*, long)"
Z128 = "void gpk::k_sweep_z<double, 7, true, false, 0>(gpk::VecOf<double>::T*, int)"
XIM = "void gpk::k_sweep_lines<double, 16, 8, false, 1, false, 8>(gpk::VecOf<double>::T*, long)"
XOTHER = "void gpk::k_stream_lines<double, 7, true, 2>(gpk::VecOf<double>::T*, int)"
COPY = "__amd_rocclr_copyBuffer"


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, (name, val) in enumerate(rows):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 64, 1, name, 64, 0, 0, 8, 0, 8, counter, val, 0, 1])


def test_classify():
    assert profiling.classify(X128) == ("x_sweep", "c128", True)
    assert profiling.classify(Y128) == ("y_sweep", "c128", True)
    assert profiling.classify(Z128) == ("z_sweep", "c128", True)
    assert profiling.classify(XIM) == ("x_sweep", "c128", False)
    assert profiling.classify("void gpk::k_sweep_z<float, 14, true, false, 0>(x)") == ("z_sweep", "c64", True)
    assert profiling.classify(XOTHER) == ("x_sweep", "c128", True)
    assert profiling.classify("void gpk::k_stream_yz<float, 5, 7, true, false, 0, 16>(x)")[0] == "yz_fused"
    assert profiling.classify(COPY) is None
    assert profiling.in_mapping(X128, [16, 8, 16, 4, 64, 7])
    assert not profiling.in_mapping(X128, [16, 4, 16, 4, 64, 7])
    assert profiling.in_mapping(Y128, [16, 8, 16, 4, 64, 7])
    assert profiling.in_mapping(Z128, [16, 8, 16, 4, 64, 7])
    assert not profiling.in_mapping(XOTHER, [16, 8, 16, 4, 64, 7])


def test_traffic_scaling(tmp_path):
    # the 1 GiB copies read 1 GiB but FETCH_SIZE counts half of it (as measured on gfx950),
    # a small copy of the same kernel does not calibrate;
    # the sweeps: x reads 10% more than psi, y and z exactly psi
    gib_kib = (1 << 30) / 1024
    npts = 8 * 6 * 4
    psi_kib = 16 * npts / 1024
    f, w, b = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "b.json"
    write_csv(f, "FETCH_SIZE", [(COPY, 3.0), (COPY, gib_kib / 2), (COPY, gib_kib / 2), (X128, 1.1 * psi_kib / 2),
                                (X128, 1.1 * psi_kib / 2), (Y128, psi_kib / 2), (Z128, psi_kib / 2),
                                (XIM, 5 * psi_kib), (XOTHER, psi_kib / 2)])
    write_csv(w, "WRITE_SIZE", [(COPY, 0.5), (COPY, gib_kib), (COPY, gib_kib), (X128, psi_kib), (X128, psi_kib),
                                (Y128, psi_kib), (Z128, psi_kib), (XIM, 5 * psi_kib), (XOTHER, psi_kib)])
    b.write_text("log line\n" + json.dumps({"dtype": "f64", "config": {"grid": [8, 6, 4], "workload": "t",
                                                                         "mapping": [16, 8, 16, 4, 64, 7]}}))
    r = profiling.traffic(str(f), str(w), str(b))
    assert r["calibration"]["dispatches"] == 2
    assert abs(r["calibration"]["fetch_scale"] - 2.0) < 1e-12
    assert abs(r["calibration"]["write_scale"] - 1.0) < 1e-12
    e = r["c128"]
    alg = 2 * 16 * npts
    assert e["algorithmic_bytes"] == alg
    assert abs(e["x_sweep"] - 2.1 * 16 * npts) < 1e-6
    assert abs(e["y_sweep"] - alg) < 1e-6 and abs(e["z_sweep"] - alg) < 1e-6
    assert abs(e["detail"]["x_sweep"]["traffic_over_algorithmic"] - 1.05) < 1e-12
    assert e["detail"]["x_sweep"]["dispatches"] == 2
    # the imaginary-time kernel is not a timed real-time sweep; the streaming one is listed apart
    assert [d["kernel"] for d in e["other"]] == ["gpk::k_stream_lines<double, 7, true, 2>"]
    assert "c64" not in r


def test_stats_table(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow([Z128, 10, 7000000, 700000, 60.0, 1, 1, 0])
        w.writerow([COPY, 2, 400000, 200000, 40.0, 1, 1, 0])
    t = profiling.stats_table(str(p), points=110100480)
    lines = t.splitlines()
    assert lines[2].startswith("| `gpk::k_sweep_z<double, 7, true, false, 0>` | 10 | 700.0 | 60.0% | 5033 |")
    assert lines[3].endswith("| 40.0% |  |")


def test_counter_table(tmp_path):
    f = tmp_path / "c.csv"
    with open(f, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEAD)
        w.writerow([0, 0, "Agent 1", 1, 1, 1, 64, 1, X128, 64, 0, 0, 8, 0, 8, "TCP_UTCL1_REQUEST_sum", 10, 0, 1])
        w.writerow([1, 1, "Agent 1", 1, 1, 1, 64, 1, X128, 64, 0, 0, 8, 0, 8, "TCP_UTCL1_REQUEST_sum", 30, 0, 1])
        w.writerow([2, 2, "Agent 1", 1, 1, 1, 64, 1, COPY, 64, 0, 0, 8, 0, 8, "TCP_UTCL1_REQUEST_sum", 5, 0, 1])
    t = profiling.counter_table([str(f)]).splitlines()
    assert t[0] == "| kernel | dispatches | TCP_UTCL1_REQUEST_sum |"
    assert t[2] == "| `gpk::k_sweep_lines<double, 16, 8, true, 2, false, 8>` | 2 | 20 |"
    assert len(t) == 3   # the copy kernel is not a sweep
    assert len(profiling.counter_table([str(f)], kernels=["rocclr"]).splitlines()) == 3
