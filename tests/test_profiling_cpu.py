"""The rocprofv3 summaries in profiling.py, on small synthetic outputs: the
kernel-trace table from a rocpd-style database (with the warm-up left out),
the traffic figure from two counter CSVs scaled by the copy kernel's
reading, and the counter table with its ratios."""
import csv
import json
import os
import sqlite3

from paper_1810_06800_amd import profiling

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
PERSISTENT = "void rsa::rsa_persistent<1, 1, false, false>(rsa::KernelArgs)"
COPY = "void at::native::elementwise_kernel<128, 2>(int, float)"


def write_counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(COLS)
        for disp, name, value in rows:
            # two TCC channels per dispatch: the summary adds them
            for half in (0.5, 0.5):
                w.writerow([disp, disp, "Agent 1", 4, 1, 1, 131072, 8, name, 128, 512, 0, 88, 0, 112, counter,
                            value * half, 0, 1])


def test_traffic_scales_each_counter_by_the_copy(tmp_path):
    copy_mib = 64
    copy_kib = copy_mib * 1024
    # FETCH_SIZE reads half of the copy's bytes, WRITE_SIZE all of them
    write_counters(str(tmp_path / "f"), "FETCH_SIZE",
                   [(1, "rsa::rsa_reset_queues(unsigned int*, unsigned int)", 2.0), (2, PERSISTENT, 1000.0),
                    (3, COPY, copy_kib / 2)])
    write_counters(str(tmp_path / "w"), "WRITE_SIZE", [(2, PERSISTENT, 300.0), (3, COPY, copy_kib)])
    out = profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "plain_scale", copy_mib, "cmd")
    assert out["FETCH_SIZE"]["scale"] == 2.0 and out["WRITE_SIZE"]["scale"] == 1.0
    assert out["FETCH_SIZE"]["dispatches"] == 1 and out["WRITE_SIZE"]["dispatches"] == 1
    assert out["bytes_per_launch"] == (1000.0 * 2.0 + 300.0) * 1024
    assert out["kernel_digest"] == profiling.kernel_digest()
    json.dumps(out)


def test_trace_summary_from_database(tmp_path):
    db = tmp_path / "run" / "trace_results.db"
    db.parent.mkdir()
    con = sqlite3.connect(str(db))
    con.execute("create table kernels (name text, duration integer, grid_x integer, workgroup_x integer, "
                "lds_size integer, vgpr_count integer, sgpr_count integer)")
    for d in (36_000_000, 38_000_000, 40_000_000):
        con.execute("insert into kernels values (?, ?, ?, ?, ?, ?, ?)", (PERSISTENT, d, 131072, 128, 31904, 88, 112))
    con.execute("insert into kernels values (?, ?, ?, ?, ?, ?, ?)",
                ("rsa::rsa_reset_queues(unsigned int*, unsigned int)", 4000, 256, 256, 0, 4, 16))
    con.commit()
    con.close()
    text = profiling.trace_summary(str(tmp_path / "run"), "t", "cmd")
    row = [l for l in text.splitlines() if "rsa_persistent" in l][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "3" and cells[2] == "38.000" and cells[3] == "36.000" and cells[4] == "40.000"
    assert cells[6:] == ["131072", "128", "31904", "88", "112"]


def test_trace_summary_skips_the_warmup_by_start_time(tmp_path):
    db = tmp_path / "run" / "trace_results.db"
    db.parent.mkdir()
    con = sqlite3.connect(str(db))
    con.execute("create table kernels (start integer, name text, duration integer, grid_x integer, "
                "workgroup_x integer, lds_size integer, vgpr_count integer, sgpr_count integer)")
    # inserted out of order: the earliest dispatch (the warm-up) is the slow one
    for start, d in ((300, 20_000_000), (100, 90_000_000), (200, 10_000_000)):
        con.execute("insert into kernels values (?, ?, ?, ?, ?, ?, ?, ?)", (start, PERSISTENT, d, 16384, 512, 0, 1, 1))
    con.commit()
    con.close()
    text = profiling.trace_summary(str(tmp_path / "run"), "t", "cmd", skip=1)
    row = [l for l in text.splitlines() if "rsa_persistent" in l][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "2" and cells[2] == "15.000" and cells[3] == "10.000" and cells[4] == "20.000"
    assert "left out" in text


def test_counter_summary_ratios(tmp_path):
    write_counters(str(tmp_path / "a"), "SQ_WAVE_CYCLES", [(2, PERSISTENT, 1000.0), (3, COPY, 5.0)])
    write_counters(str(tmp_path / "b"), "SQ_WAIT_ANY", [(2, PERSISTENT, 250.0)])
    write_counters(str(tmp_path / "c"), "TCC_HIT_sum", [(2, PERSISTENT, 30.0)])
    write_counters(str(tmp_path / "d"), "TCC_REQ_sum", [(2, PERSISTENT, 40.0)])
    text = profiling.counter_summary([str(tmp_path / x) for x in "abcd"], "w", "cmd")
    assert "| `SQ_WAVE_CYCLES` | 1000 |" in text
    assert "| cycles a wave waits (any), % of wave-cycles | 25 |" in text
    assert "| L2 hit rate, % | 75 |" in text
