"""Host logic of the rocprofv3 summariser: copy-probe calibration of the HBM
byte counters and the instruction-issue table, on synthetic CSV files."""
import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
COPY = "k_copy_probe(uint4 const*, uint4*, long)"
STEP = "void mclbm::k_step<float, 8, 0, 0, false>(mclbm::Inst, int, mclbm::Fields, double*)"


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COLS)
        w.writeheader()
        for disp, (name, grid, counter, value, t0, t1) in enumerate(rows):
            r = {c: 0 for c in COLS}
            r.update(Dispatch_Id=disp // 8 + 1, Kernel_Name=name, Grid_Size=grid, Counter_Name=counter,
                     Counter_Value=value, Start_Timestamp=t0, End_Timestamp=t1)
            w.writerow(r)


def _agent(path):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Num_Xcc", "Cu_Count"])
        w.writeheader()
        w.writerow({"Name": "gfx950", "Num_Xcc": 8, "Cu_Count": 256})


def test_summary_calibration_and_issue_table(tmp_path):
    st, fe, wr, iss = (tmp_path / d for d in ("stats", "fetch", "write", "issue"))
    for d in (st, fe, wr, iss):
        d.mkdir()
    with open(st / "s_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": STEP, "Calls": 10, "AverageNs": 650000.0, "Percentage": 90.0})
        w.writerow({"Name": COPY, "Calls": 2, "AverageNs": 700000.0, "Percentage": 10.0})
    grid = 1 << 20                       # copy probe: 16 B per lane each way
    true_bytes = grid * 16
    # the copy probe's FETCH_SIZE reads half its true bytes, WRITE_SIZE all of them
    _counters(fe / "f_counter_collection.csv", [(COPY, grid, "FETCH_SIZE", true_bytes / 2048, 0, 1),
                                                 (STEP, 4096, "FETCH_SIZE", 1000.0, 0, 1)])
    _counters(wr / "w_counter_collection.csv", [(COPY, grid, "WRITE_SIZE", true_bytes / 1024, 0, 1),
                                                 (STEP, 4096, "WRITE_SIZE", 3000.0, 0, 1)])
    # one 100 us dispatch of 1000 waves at 2.0 GHz issuing 25.6 M VALU instructions:
    # 256 CUs x 200,000 cycles = 51.2 M issue slots, half used
    t0, t1 = 1_000_000, 1_100_000
    _counters(iss / "i_counter_collection.csv", [
        (STEP, 4096, "SQ_WAVES", 1000, t0, t1), (STEP, 4096, "SQ_INSTS_VALU", 25.6e6, t0, t1),
        (STEP, 4096, "SQ_INSTS_SALU", 300000, t0, t1), (STEP, 4096, "SQ_INSTS_LDS", 30000, t0, t1),
        (STEP, 4096, "SQ_INSTS_VMEM_RD", 27500, t0, t1), (STEP, 4096, "SQ_INSTS_VMEM_WR", 18000, t0, t1),
        (STEP, 4096, "GRBM_GUI_ACTIVE", 8 * 200000, t0, t1)])
    _agent(iss / "i_agent_info.csv")
    out = tmp_path / "sum.md"
    subprocess.run([sys.executable, "-m", "paper_2009_12584_amd.rocprof_summary", "--stats", str(st), "--fetch",
                    str(fe), "--write", str(wr), "--issue", str(iss), "--kernel-hash", "abc", "--out", str(out)],
                   check=True, cwd=ROOT, capture_output=True)
    text = out.read_text()
    assert "kernel source hash: `abc`" in text
    assert "factor 2.000" in text and "factor 1.000" in text
    # step: 1000 KiB x 2 fetched, 3000 KiB x 1 written
    assert "| k_step<float, 8, 0, 0, false> | %.3f | %.3f | %.3f |" % (2048000 / 1e6, 3072000 / 1e6,
                                                                       5120000 / 1e6) in text
    row = [l for l in text.splitlines() if l.startswith("| k_step<float, 8, 0, 0, false> | 1000 |")]
    assert row, text
    cells = [c.strip() for c in row[0].strip("|").split("|")]
    assert cells[2] == "25600" and cells[3] == "300" and cells[7] == "100.0"
    assert cells[8] == "2.00" and cells[9] == "0.50"
