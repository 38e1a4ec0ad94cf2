"""rocprofv3 summaries of the library's kernels (run where the GPU is).

Commands (from the repository root):

  python -m paper_1810_06800_amd.profiling workload NAME [--copy-mib M]
      one batch of a named workload through the C ABI, then an elementwise
      copy of M MiB (read M, write M) whose counter readings calibrate the
      byte counters; run it under ``rocprofv3 --pmc FETCH_SIZE`` and again
      under ``rocprofv3 --pmc WRITE_SIZE``

  python -m paper_1810_06800_amd.profiling trace-summary OUT_DIR --title T --cmd C [--skip N]
      markdown table of a ``rocprofv3 --kernel-trace --stats`` run (calls,
      average / min / max duration, launch shape) from its output directory;
      --skip drops each kernel's first N dispatches (the benchmark's warm-up)

  python -m paper_1810_06800_amd.profiling counters DIR [DIR ...] --workload NAME --cmd C
      markdown table of ``rocprofv3 --pmc`` runs of the workload program: every
      counter's value for the persistent kernel's dispatch, and the ratios read
      from them (instruction mix, cycles waiting, L2 hit rate)

  python -m paper_1810_06800_amd.profiling traffic --fetch DIR --write DIR --workload NAME --cmd C
      HBM bytes per launch of the persistent kernel from the two counter
      runs, each scaled by what the same counter reads for the copy kernel
      of known size; JSON with the digest of the kernel source it was taken on

The counters are per dispatch and summed over the L2 (TCC) channels, in KiB.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# the kernel sources and the autotune table (which picks the tile a workload runs with)
KERNEL_SOURCES = ["paper_1810_06800_amd/csrc/rsa_kernels.hip", "paper_1810_06800_amd/csrc/rsa_device.h",
                  "paper_1810_06800_amd/tiles.json"]
PERSISTENT = "rsa_persistent"


def kernel_digest() -> str:
    """sha256 prefix of the kernel sources and the tile table (counter
    readings are tied to it)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# the profiled program
# ---------------------------------------------------------------------------

def run_workload(name: str, copy_mib: int) -> None:
    import torch

    from . import rsa, workloads

    descs = workloads.CONFIGS[name]()
    ctx = rsa.Context(0)
    print(f"# workload {name}: {len(descs)} samples", flush=True)
    res = ctx.run(descs)
    bad = sum(r["status"] != 0 for r in res)
    print(f"# workload done, {sum(r['n_jam'] for r in res)} deposits, {bad} failed", flush=True)
    ctx.close()
    n = copy_mib * (1 << 20) // 4
    src = torch.empty(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)   # reads and writes copy_mib MiB
    torch.cuda.synchronize()
    print(f"# copy of {copy_mib} MiB done", flush=True)
    if bad:
        sys.exit(1)


# ---------------------------------------------------------------------------
# reading rocprofv3 output (rocpd database or CSV)
# ---------------------------------------------------------------------------

def _find(out_dir: str, pattern: str):
    return sorted(glob.glob(os.path.join(out_dir, "**", pattern), recursive=True))


def kernel_rows(out_dir: str):
    """(name, duration_ns, grid, workgroup, lds, vgpr, sgpr) per dispatch, in
    order of start time."""
    rows = []
    for db in _find(out_dir, "*.db"):
        con = sqlite3.connect(db)
        cols = "name, duration, grid_x, workgroup_x, lds_size, vgpr_count, sgpr_count from kernels"
        try:
            try:
                cur = con.execute("select start, " + cols)
            except sqlite3.OperationalError:   # no start column: rows in insertion order
                cur = con.execute("select rowid, " + cols)
            rows.extend(tuple(r) for r in cur)
        finally:
            con.close()
    if not rows:
        for path in _find(out_dir, "*kernel_trace.csv"):
            with open(path) as f:
                for r in csv.DictReader(f):
                    rows.append((int(r["Start_Timestamp"]), r["Kernel_Name"],
                                 int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                                 int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0),
                                 int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 0),
                                 int(r.get("LDS_Block_Size") or r.get("Lds_Size") or 0),
                                 int(r.get("VGPR_Count") or 0), int(r.get("SGPR_Count") or 0)))
    rows.sort(key=lambda r: r[0])
    return [r[1:] for r in rows]


def counter_rows(out_dir: str, counter: str):
    """(dispatch id, kernel name, grid, value) of one counter, summed per dispatch."""
    acc = {}
    for path in _find(out_dir, "*counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                key = (int(r["Dispatch_Id"]), r["Kernel_Name"], int(r.get("Grid_Size") or 0))
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    if not acc:
        for db in _find(out_dir, "*.db"):
            con = sqlite3.connect(db)
            try:
                q = ("select dispatch_id, kernel_name, grid_size, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id")
                for d, name, grid, v in con.execute(q, (counter,)):
                    acc[(int(d), name, int(grid or 0))] = float(v)
            finally:
                con.close()
    return [(d, name, grid, v) for (d, name, grid), v in sorted(acc.items())]


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def trace_summary(out_dir: str, title: str, cmd: str, skip: int = 0) -> str:
    rows = kernel_rows(out_dir)
    if not rows:
        raise SystemExit(f"no kernel trace under {out_dir}")
    groups = {}
    for name, dur, grid, wg, lds, vgpr, sgpr in rows:
        g = groups.setdefault(short(name), {"d": [], "n": 0, "shape": (grid, wg, lds, vgpr, sgpr)})
        g["n"] += 1
        if g["n"] > skip:   # the first `skip` dispatches of each kernel are the warm-up
            g["d"].append(dur)
    groups = {k: g for k, g in groups.items() if g["d"]}
    total = sum(sum(g["d"]) for g in groups.values())
    out = [f"# {title}", "", "command (from the repository root, one MI355X):", "", f"    {cmd}", ""]
    if skip:
        out += [f"The first {skip} dispatch(es) of each kernel (the warm-up) are left out.", ""]
    out += ["| kernel | calls | avg ms | min ms | max ms | total % | grid (threads) | workgroup | LDS B | VGPR | SGPR |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["d"])):
        d = g["d"]
        grid, wg, lds, vgpr, sgpr = g["shape"]
        out.append(f"| `{name}` | {len(d)} | {sum(d) / len(d) / 1e6:.3f} | {min(d) / 1e6:.3f} | "
                   f"{max(d) / 1e6:.3f} | {100 * sum(d) / total:.2f} | {grid} | {wg} | {lds} | {vgpr} | {sgpr} |")
    return "\n".join(out) + "\n"


def traffic(fetch_dir: str, write_dir: str, workload: str, copy_mib: int, cmd: str) -> dict:
    copy_bytes = copy_mib * (1 << 20)
    out = {"workload": workload, "kernel": PERSISTENT, "kernel_digest": kernel_digest(), "command": cmd,
           "copy_bytes": copy_bytes}
    total = 0.0
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = counter_rows(d, counter)
        ours = [r for r in rows if PERSISTENT in r[1]]
        copies = [r for r in rows if PERSISTENT not in r[1] and "rsa_" not in r[1]]
        if not ours or not copies:
            raise SystemExit(f"{counter}: missing dispatches under {d} ({len(ours)} ours, {len(copies)} others)")
        copy_kib = max(copies, key=lambda r: r[3])[3]
        scale = copy_bytes / (copy_kib * 1024.0)
        ours_kib = sum(r[3] for r in ours)
        nbytes = ours_kib * 1024.0 * scale
        out[counter] = {"kernel_kib": ours_kib, "dispatches": len(ours), "copy_kib": copy_kib,
                        "scale": scale, "bytes": nbytes}
        total += nbytes
    out["bytes_per_launch"] = total
    return out


# ratios read from the counter table: (label, numerator, denominator, scale)
RATIOS = [
    ("VALU instructions per wave-cycle", "SQ_INSTS_VALU", "SQ_WAVE_CYCLES", 1.0),
    ("cycles a wave waits (any), % of wave-cycles", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES", 100.0),
    ("cycles a wave waits for an instruction to issue, % of wave-cycles", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES",
     100.0),
    ("cycles with a VALU instruction in flight, % of wave-cycles", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", 100.0),
    ("cycles with a vector memory instruction in flight, % of wave-cycles", "SQ_ACTIVE_INST_VMEM",
     "SQ_WAVE_CYCLES", 100.0),
    ("cycles with an LDS instruction in flight, % of wave-cycles", "SQ_ACTIVE_INST_LDS", "SQ_WAVE_CYCLES", 100.0),
    ("L2 hit rate, %", "TCC_HIT_sum", "TCC_REQ_sum", 100.0),
    ("L2 requests per vector memory instruction", "TCC_REQ_sum", "SQ_INSTS_VMEM", 1.0),
]


def counter_summary(dirs, workload: str, cmd: str) -> str:
    """Every counter of the persistent kernel's dispatch(es) over the given
    runs, and the ratios of RATIOS that the runs cover."""
    vals = {}
    for d in dirs:
        names = set()
        for path in _find(d, "*counter_collection.csv"):
            with open(path) as f:
                for r in csv.DictReader(f):
                    names.add(r["Counter_Name"])
        for name in sorted(names):
            rows = [r for r in counter_rows(d, name) if PERSISTENT in r[1]]
            if rows:
                vals[name] = sum(r[3] for r in rows)
    if not vals:
        raise SystemExit("no counters of the persistent kernel found")
    out = [f"# rsa_persistent counters, workload {workload}", "",
           "command per pass (from the repository root, one MI355X; COUNTERS is one line of the table's",
           "passes):", "", f"    {cmd}", "", "| counter | value |", "|---|---|"]
    for name in sorted(vals):
        out.append(f"| `{name}` | {vals[name]:.6g} |")
    out += ["", "| ratio | value |", "|---|---|"]
    for label, num, den, scale in RATIOS:
        if num in vals and den in vals and vals[den]:
            out.append(f"| {label} | {scale * vals[num] / vals[den]:.4g} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1810_06800_amd.profiling")
    sub = ap.add_subparsers(dest="action", required=True)
    w = sub.add_parser("workload")
    w.add_argument("name")
    w.add_argument("--copy-mib", type=int, default=2048)
    t = sub.add_parser("trace-summary")
    t.add_argument("out_dir")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--skip", type=int, default=0)
    cs = sub.add_parser("counters")
    cs.add_argument("dirs", nargs="+")
    cs.add_argument("--workload", required=True)
    cs.add_argument("--cmd", required=True)
    tr = sub.add_parser("traffic")
    tr.add_argument("--fetch", required=True)
    tr.add_argument("--write", required=True)
    tr.add_argument("--workload", required=True)
    tr.add_argument("--copy-mib", type=int, default=2048)
    tr.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.action == "workload":
        run_workload(a.name, a.copy_mib)
    elif a.action == "trace-summary":
        sys.stdout.write(trace_summary(a.out_dir, a.title, a.cmd, a.skip))
    elif a.action == "counters":
        sys.stdout.write(counter_summary(a.dirs, a.workload, a.cmd))
    else:
        print(json.dumps(traffic(a.fetch, a.write, a.workload, a.copy_mib, a.cmd), indent=1))


if __name__ == "__main__":
    main()
