"""Turn two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE; CSV output) into HBM bytes per
launch of one kernel, calibrated against a plain device copy of known size recorded in the
same runs (the bench's --copy-calibration-mb option).

usage: python -m paper_1906_07925_amd.traffic <fetch.csv> <write.csv> <kernel> <copy_MiB> <out.json> <command>
       <bench output of the counter run>
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


if __name__ == "__main__":
    main()
