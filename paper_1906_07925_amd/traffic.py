"""Turn two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE; CSV output) into HBM bytes per
launch of one kernel, calibrated against a plain device copy of known size recorded in the
same runs (the bench's --copy-calibration-mb option).

usage: python -m paper_1906_07925_amd.traffic <fetch.csv> <write.csv> <kernel> <copy_MiB> <out.json> <command>
       <bench output of the counter run>
       python -m paper_1906_07925_amd.traffic step <fetch.csv> <write.csv> <copy_MiB> <steps> <title> <command>
       <note> <out.md>      (every kernel of the run, per step, and the whole-step total)
The bench output (its JSON line) gives the cell size and lanes per particle of the run.
"""
from __future__ import annotations

import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def per_dispatch(path: str, counter: str):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def calibration(rows, copy_bytes: int) -> float:
    """true bytes / counted bytes for the largest device copy in the run."""
    copies = [v for k, g, v in rows if "copyBuffer" in k]
    if not copies:
        raise SystemExit("no copy kernel in the run")
    counted = max(copies) * 1024.0
    return copy_bytes / counted


def main():
    fetch_csv, write_csv, kernel, copy_mib, out, command, bench_out = sys.argv[1:8]
    cfg = None
    for line in open(bench_out):
        line = line.strip()
        if line.startswith("{") and '"metric"' in line:
            cfg = json.loads(line)["config"]
    if cfg is None:
        raise SystemExit("no benchmark line in " + bench_out)
    copy_bytes = int(copy_mib) << 20
    f = per_dispatch(fetch_csv, "FETCH_SIZE")
    w = per_dispatch(write_csv, "WRITE_SIZE")
    cf, cw = calibration(f, copy_bytes), calibration(w, copy_bytes)
    fk = [v for k, g, v in f if kernel in k]
    wk = [v for k, g, v in w if kernel in k]
    fetch = cf * 1024.0 * sum(fk) / len(fk)
    write = cw * 1024.0 * sum(wk) / len(wk)
    sys.path.insert(0, ROOT)
    import bench
    rec = {"kernel": kernel, "workload": bench.WORKLOAD, "kernel_source_digest": bench.kernel_source_digest(),
           "cell_log2": cfg["cell_log2"], "lanes": cfg["lanes"],
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write, "fetch_scale": cf, "write_scale": cw,
           "launches": len(fk), "command": command}
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec))


def step_table(fetch_csv: str, write_csv: str, copy_mib: int, steps: int, title: str, command: str,
               note: str) -> str:
    """Markdown table of the calibrated HBM bytes of every kernel of a counter run, summed over
    its launches and divided by the run's step count, with the whole-step total."""
    import collections
    copy_bytes = int(copy_mib) << 20
    f = per_dispatch(fetch_csv, "FETCH_SIZE")
    w = per_dispatch(write_csv, "WRITE_SIZE")
    cf, cw = calibration(f, copy_bytes), calibration(w, copy_bytes)
    acc = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for k, g, v in f:
        if "copyBuffer" in k or "fillBuffer" in k or "at::" in k:
            continue
        name = k.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        acc[name][0] += 1
        acc[name][1] += cf * 1024.0 * v
    for k, g, v in w:
        if "copyBuffer" in k or "fillBuffer" in k or "at::" in k:
            continue
        name = k.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        acc[name][2] += cw * 1024.0 * v
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "", note, "",
           f"Calibration (a {copy_mib} MiB device copy in the same runs): fetch scale {cf:.4f}, write scale {cw:.4f}.",
           "", "| kernel | launches | MB read / step | MB written / step |", "|---|---|---|---|"]
    tr = tw = 0.0
    for name, (nl, fb, wb) in sorted(acc.items(), key=lambda kv: -(kv[1][1] + kv[1][2])):
        out.append(f"| {name} | {nl} | {fb / steps / 1e6:.1f} | {wb / steps / 1e6:.1f} |")
        tr += fb
        tw += wb
    out.append(f"| **step total** | | **{tr / steps / 1e6:.1f}** | **{tw / steps / 1e6:.1f}** |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "step":
        fetch_csv, write_csv, copy_mib, steps, title, command, note, dest = sys.argv[2:10]
        open(dest, "w").write(step_table(fetch_csv, write_csv, int(copy_mib), int(steps), title, command, note))
    else:
        main()
