"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_2004_11227_amd.profiling KTRACE_DIR FETCH_DIR WRITE_DIR OUT_PREFIX KERNEL_SUBSTR
        [--copy-bytes N] [--launch-bytes N] [--command "..."]

KTRACE_DIR holds `*_kernel_stats.csv` of a `--kernel-trace --stats` run;
FETCH_DIR / WRITE_DIR hold `*_counter_collection.csv` of `--pmc FETCH_SIZE` /
`--pmc WRITE_SIZE` runs of a program that first copies COPY_BYTES with a
plain copy kernel (the counter calibration) and then runs the kernel of
interest.  Writes OUT_PREFIX.md (human summary) and OUT_PREFIX_traffic.json
(per-launch HBM bytes of the kernel of interest, scaled by the copy
calibration, with the source hash of the kernel it was measured on).
With FETCH_DIR and WRITE_DIR given as `-`, only the kernel-trace table is
written (OUT_PREFIX.md); if KTRACE_DIR also holds the per-dispatch
`*_kernel_trace.csv`, the dispatches of the kernel of interest are split by
grid size, and launches that returned at once on the solver's done flag
(under a tenth of their grid's median) are counted apart, so that one
workload's average can be read off a program that runs several.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def _one(pattern):
    files = glob.glob(pattern, recursive=True)
    if not files:
        raise FileNotFoundError(pattern)
    return files[0]


def kernel_stats(d):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_stats.csv")))))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["Percentage"])) for r in rows]


def dispatches_by_grid(d, kernel):
    """{grid work-items: [durations ns]} of the dispatches whose name holds
    `kernel`, from a per-dispatch kernel trace (None when absent)."""
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        return None
    out = {}
    for r in csv.DictReader(open(files[0])):
        if kernel not in r["Kernel_Name"]:
            continue
        if "Grid_Size" in r:
            g = int(r["Grid_Size"])
        else:
            g = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y", 1) or 1) * int(r.get("Grid_Size_Z", 1) or 1)
        out.setdefault(g, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def grid_table(by_grid):
    lines = ["", "Dispatches of the kernel of interest by grid size (launches under a tenth of their grid's "
             "median are early exits on the done flag):", "",
             "| grid work-items | workgroups of 256 | dispatches | early exits | average us (full) | "
             "median us (full) |", "|---|---|---|---|---|---|"]
    for g in sorted(by_grid, reverse=True):
        ds = sorted(by_grid[g])
        med = ds[len(ds) // 2]
        full = [x for x in ds if x >= 0.1 * med]
        lines.append(f"| {g} | {g // 256} | {len(ds)} | {len(ds) - len(full)} | "
                     f"{sum(full) / len(full) / 1e3:.2f} | {full[len(full) // 2] / 1e3:.2f} |")
    return lines


def counter_table(dirs, kernel):
    """Per-dispatch averages of every counter collected in `dirs` for the
    kernel of interest, with the ratios read off them."""
    agg = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if kernel in r["Kernel_Name"]:
                    agg.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {k: sum(v) / len(v) for k, v in agg.items()}
    lines = ["", "## Instruction and wait counters (--pmc, one pass per group; per dispatch)", "",
             "| counter | average per dispatch |", "|---|---|"]
    for k in sorted(avg):
        lines.append(f"| {k} | {avg[k]:.0f} |")
    w = avg.get("SQ_WAVES")
    if w:
        lines += ["", "Per wave: " + ", ".join(f"{k[9:] if k.startswith('SQ_INSTS_') else k} {avg[k] / w:.0f}"
                                           for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
                                                     "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR") if k in avg) + "."]
    if "SQ_LDS_BANK_CONFLICT" in avg and avg.get("SQ_ACTIVE_INST_LDS"):
        lines.append(f"LDS bank-conflict cycles per LDS-active cycle: "
                     f"{avg['SQ_LDS_BANK_CONFLICT'] / avg['SQ_ACTIVE_INST_LDS']:.2f}.")
    if avg.get("SQ_WAVE_CYCLES"):
        for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS"):
            if k in avg:
                lines.append(f"{k} / SQ_WAVE_CYCLES: {avg[k] / avg['SQ_WAVE_CYCLES']:.2f}.")
    return lines


def counters(d):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))))
    agg = {}
    for r in rows:
        agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in agg.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("ktrace")
    ap.add_argument("fetch")
    ap.add_argument("write")
    ap.add_argument("out")
    ap.add_argument("kernel")
    ap.add_argument("--copy-bytes", type=int, default=256 << 20)
    ap.add_argument("--launch-bytes", type=int, default=0)
    ap.add_argument("--command", default="")
    ap.add_argument("--sources", nargs="*", default=[])
    ap.add_argument("--pmc-dirs", nargs="*", default=[],
                    help="directories of further --pmc runs (SQ_ counters) of the same program")
    a = ap.parse_args()
    ks = kernel_stats(a.ktrace)
    if a.fetch == "-" and a.write == "-":
        total = sum(calls * avg for _, calls, avg, _ in ks)
        lines = [f"# rocprofv3 kernel trace: {a.kernel}", "", f"Command: `{a.command}`", "",
                 "| kernel | calls | average us | % time |", "|---|---|---|---|"]
        for name, calls, avg, pct in ks[:16]:
            lines.append(f"| `{name[:110]}` | {calls} | {avg / 1e3:.2f} | {pct:.2f} |")
        lines += ["", f"Total kernel time {total / 1e6:.1f} ms over {sum(c for _, c, _, _ in ks)} dispatches."]
        by_grid = dispatches_by_grid(a.ktrace, a.kernel)
        if by_grid:
            lines += grid_table(by_grid)
        open(a.out + ".md", "w").write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    fe, wr = counters(a.fetch), counters(a.write)
    copy_k = [k for k in fe if "copyBuffer" in k or "copy" in k.lower()]
    ck = copy_k[0]
    exp_kib = a.copy_bytes / 1024.0
    f_fetch = exp_kib / fe[ck][1]
    f_write = exp_kib / wr[ck][1]
    kk = [k for k in fe if a.kernel in k]
    target = kk[0]
    fetch_b = fe[target][1] * 1024.0 * f_fetch
    write_b = wr[target][1] * 1024.0 * f_write
    lines = [f"# rocprofv3 summary: {a.kernel}", "", f"Command: `{a.command}`", "",
             "## Kernel trace (--kernel-trace --stats)", "",
             "| kernel | calls | average us | % time |", "|---|---|---|---|"]
    for name, calls, avg, pct in ks[:12]:
        lines.append(f"| `{name[:110]}` | {calls} | {avg / 1e3:.2f} | {pct:.2f} |")
    lines += ["", "## HBM traffic (--pmc FETCH_SIZE, --pmc WRITE_SIZE; KiB per dispatch)", "",
              f"Calibration: copy kernel `{ck[:60]}` of {a.copy_bytes} B read + write: "
              f"FETCH_SIZE {fe[ck][1]:.0f} KiB (factor {f_fetch:.3f}), WRITE_SIZE {wr[ck][1]:.0f} KiB "
              f"(factor {f_write:.3f}).", "",
              "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|---|"]
    for k in fe:
        lines.append(f"| `{k[:110]}` | {fe[k][0]} | {fe[k][1]:.1f} | {wr.get(k, (0, 0))[1]:.1f} |")
    lines += ["", f"Kernel of interest `{target[:100]}`: calibrated traffic per launch "
              f"{fetch_b / 1e6:.2f} MB read + {write_b / 1e6:.2f} MB written = {(fetch_b + write_b) / 1e6:.2f} MB"]
    if a.launch_bytes:
        lines.append(f"(algorithmic {a.launch_bytes / 1e6:.2f} MB per launch; ratio "
                     f"{(fetch_b + write_b) / a.launch_bytes:.3f})")
    if a.pmc_dirs:
        lines += counter_table(a.pmc_dirs, a.kernel)
    open(a.out + ".md", "w").write("\n".join(lines) + "\n")
    json.dump({"kernel": target, "kernel_hash": source_hash(a.sources) if a.sources else None,
               "bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b, "write_bytes": write_b,
               "fetch_factor": f_fetch, "write_factor": f_write, "command": a.command},
              open(a.out + "_traffic.json", "w"), indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
