"""The rocprofv3 summariser on small synthetic CSVs: interval unions, the timed window found by
counting theta dispatches, the copy-calibrated HBM bytes per counted Jacobi launch, and the
MFMA utilisation and instruction mix from SQ counters."""

import csv
import json

from paper_2312_02667_amd import trace_summary as ts

TRACE_COLS = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id",
              "Kernel_Id", "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp",
              "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
              "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z", "Grid_Size_X",
              "Grid_Size_Y", "Grid_Size_Z"]
PMC_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
            "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
            "Counter_Value", "Start_Timestamp", "End_Timestamp"]
THETA = "void ptebd::(anonymous namespace)::theta_kernel<float>(ptebd::GateDesc const*)"
JAC = ("void ptebd::(anonymous namespace)::jacobi_round_kernel<float>(ptebd::GateDesc "
       "const*, int, int, ptebd::LayerOut, double, int, double, int, int)")
WB = "void ptebd::(anonymous namespace)::writeback_kernel<float>(ptebd::GateDesc const*)"
COPY = "(anonymous namespace)::hbm_copy_kernel(HIP_vector_type<float, 4u> const*)"


def test_union_and_short_names():
    assert ts.union_ms([(0, 2_000_000), (1_000_000, 3_000_000), (5_000_000, 6_000_000)]) == 4.0
    assert ts.union_ms([]) == 0
    assert ts.short_name(JAC) == "jacobi_round_kernel<float>"
    assert ts.short_name(COPY) == "hbm_copy_kernel"


def _bench_log(path, kernels, steps=1):
    with open(path, "w") as f:
        f.write("set-up layer 1: ...\n")
        f.write(json.dumps({"steps": steps, "ms_per_step": 10.0, "kernels": kernels}) + "\n")


def test_trace_window_and_jacobi_union(tmp_path, capsys):
    rows = []

    def add(name, a, b):
        rows.append({c: 0 for c in TRACE_COLS} | {"Kernel_Name": name, "Start_Timestamp": a,
                                                   "End_Timestamp": b, "Dispatch_Id": len(rows)})
    # one set-up layer (two theta halves, one round), then the timed layer: two theta
    # halves, two overlapping half-round dispatches, a write-back
    add(THETA, 0, 10)
    add(THETA, 0, 10)
    add(JAC, 20, 30)
    add(WB, 30, 40)
    add(THETA, 1_000_000, 2_000_000)
    add(THETA, 1_000_000, 2_000_000)
    add(JAC, 2_000_000, 5_000_000)
    add(JAC, 3_000_000, 6_000_000)
    add(WB, 6_000_000, 7_000_000)
    p = tmp_path / "t.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=TRACE_COLS)
        w.writeheader()
        w.writerows(rows)
    _bench_log(tmp_path / "b.log", {"jacobi": {"total_ms": 4.0, "launches": 1}})
    ts.main(["trace", "--csv", str(p), "--bench", str(tmp_path / "b.log"), "--setup-layers",
             "1", "--breakdown"])
    out = capsys.readouterr().out
    assert "6.0 ms from the first timed theta dispatch" in out
    assert "| jacobi | 2 | 6.00 | 4.00 | 0.667 |" in out
    assert "union 4.00 ms, 4.0000 ms per counted launch (+0.0 % against the events)" in out


def test_traffic_scaled_by_the_copy(tmp_path, capsys):
    def write(path, counter, copy_kib, jac_kib):
        rows = []
        for i, (name, v) in enumerate([(COPY, copy_kib), (THETA, 1.0), (THETA, 1.0),
                                       (JAC, 999.0), (THETA, 2.0), (THETA, 2.0),
                                       (JAC, jac_kib), (JAC, jac_kib)]):
            rows.append({c: 0 for c in PMC_COLS} | {"Dispatch_Id": i + 1, "Kernel_Name": name,
                                                     "Counter_Name": counter,
                                                     "Counter_Value": v})
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=PMC_COLS)
            w.writeheader()
            w.writerows(rows)
    # the read counter reads half the copy's bytes (its unit is 2 KiB here): scale 2
    write(tmp_path / "f.csv", "FETCH_SIZE", 512.0, 100.0)
    write(tmp_path / "w.csv", "WRITE_SIZE", 1024.0, 50.0)
    _bench_log(tmp_path / "b.log", {"jacobi": {"total_ms": 1.0, "launches": 1, "bytes": 5e5},
                                    "theta": {"bytes": 1e4}})
    ts.main(["traffic", "--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
             "--bench", str(tmp_path / "b.log"), "--setup-layers", "1", "--copy-mib", "1"])
    out = capsys.readouterr().out
    # two timed dispatches, one counted launch: (2 x 100 KiB x 2 + 2 x 50 KiB) per launch
    assert f"hbm_bytes_per_launch: {(400 + 100) * 1024.0:.6e}" in out
    assert "scale factor 2.0000" in out and "scale factor 1.0000" in out
    assert len(ts.kernel_source_digest()) == 64


def test_counters_mfma_utilisation(tmp_path, capsys):
    rows = []
    # one set-up layer (two theta dispatches), then the timed layer: two theta dispatches and
    # two Jacobi dispatches of 1 ms each
    plan = [(THETA, 0, 1), (THETA, 1, 2), (THETA, 10, 11), (THETA, 11, 12),
            (JAC, 1_000_000, 2_000_000), (JAC, 2_000_000, 3_000_000)]
    for i, (name, a, b) in enumerate(plan):
        vals = {"SQ_INSTS_VALU_MFMA_MOPS_F32": 1000.0, "SQ_VALU_MFMA_BUSY_CYCLES": 1024 * 600.0,
                "GRBM_GUI_ACTIVE": 8 * 2400.0, "SQ_INSTS_VALU": 120.0, "SQ_INSTS_MFMA": 10.0,
                "SQ_INSTS_LDS": 20.0, "SQ_LDS_BANK_CONFLICT": 5.0, "SQ_LDS_IDX_ACTIVE": 50.0}
        for c, v in vals.items():
            rows.append({k: 0 for k in PMC_COLS} | {"Dispatch_Id": i + 1, "Kernel_Name": name,
                                                     "Counter_Name": c, "Counter_Value": v,
                                                     "Start_Timestamp": a, "End_Timestamp": b})
    p = tmp_path / "c.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=PMC_COLS)
        w.writeheader()
        w.writerows(rows)
    ts.main(["counters", "--csv", str(p), "--setup-layers", "1"])
    out = capsys.readouterr().out
    # busy 600 of 2400 active cycles per SIMD; 2 x 1000 x 512 flops in 2 ms
    assert "| jacobi_round | 2 | 1.0240e+06 | 0.250 |" in out
    assert "| 12.0 | 2.00 | 0.100 |" in out
