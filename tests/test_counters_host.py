"""Host logic that turns rocprofv3 FETCH_SIZE / WRITE_SIZE runs into HBM bytes
per launch (paper_1810_11765_amd/counters.py), on hand-written CSVs."""
import csv
import json

from paper_1810_11765_amd import counters

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, COLS)
        w.writeheader()
        for i, (name, grid, v) in enumerate(rows):
            w.writerow({c: 0 for c in COLS} | {"Dispatch_Id": i + 1, "Grid_Size": grid, "Kernel_Name": name,
                                                "Counter_Name": counter, "Counter_Value": v})


def test_scaled_bytes_per_launch(tmp_path):
    commit = "void k_doall<MLifeCommit>(DevHeap, unsigned int, unsigned long, MLifeCommit::Args)"
    sweep = "smmo::k_doall_axpy<4>"
    # the 1 GiB copy reads half its bytes in the fetch counter's units: factor 2
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(counters.CALIB_KERNEL, 131072, 524288.0),
                                            (counters.CALIB_KERNEL, 512, 4.0),
                                            (commit, 786432, 100.0), (commit, 786432, 300.0),
                                            (sweep, 2097152, 1000.0), (sweep, 4096, 10.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(counters.CALIB_KERNEL, 131072, 1048576.0),
                                            (commit, 786432, 50.0), (commit, 786432, 50.0),
                                            (sweep, 2097152, 500.0), (sweep, 4096, 5.0)])
    rec = counters.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    k = rec["kernels"]
    assert k["k_doall<MLifeCommit>"] == {"fetch_kib_raw": 200.0, "write_kib_raw": 50.0, "dispatches": 2,
                                         "bytes_per_launch": (2 * 200 + 50) * 1024}
    assert k["k_doall_axpy<4>@2^21"]["bytes_per_launch"] == (2 * 1000 + 500) * 1024
    assert k["k_doall_axpy<4>"]["bytes_per_launch"] == (2 * 10 + 5) * 1024
    assert not any(n.startswith("__amd") for n in k)
    assert counters.short_name("smmo::k_doall<smmo::MLifeCommit, false>", 786432) == "k_doall<MLifeCommit>"
    assert counters.short_name("smmo::k_doall<smmo::MFishPlan, false, true>", 1) == "k_doall<MFishPlan>"
    assert counters.short_name("k_destroy(DevHeap, unsigned long const*)", 1) == "k_destroy"
    assert rec["source_sha256"] == counters.kernel_source_hash()
    counters.main(["x", str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "o.json")])
    assert json.load(open(tmp_path / "o.json"))["kernels"] == k
