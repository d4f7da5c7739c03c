"""Summarise a rocprofv3 run (rocpd SQLite output) into a short markdown kernel table."""
from __future__ import annotations

import re
import sqlite3
import sys


def short_name(n: str) -> str:
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"^void\s+", "", n)
    head = n.split("(")[0]
    return head.split("::")[-1] if "::" in head and "<" not in head else head.replace("mpsph::", "")


def kernel_rows(path: str):
    """(name, calls, total us, average us, percent) from a rocpd database or a kernel_stats.csv."""
    if path.endswith(".csv"):
        import csv
        rows = []
        for r in csv.DictReader(open(path)):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
        return rows
    con = sqlite3.connect(path)
    return [(short_name(n), c, t, a, p) for n, c, t, a, p in
            con.execute("select name,total_calls,total_duration,average,percentage from top_kernels")]


def markdown(db: str, title: str, command: str, note: str) -> str:
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "", note, "",
           "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for n, c, t, a, p in kernel_rows(db):
        out.append(f"| {n} | {c} | {t:.0f} | {a:.1f} | {p:.1f} |")
    return "\n".join(out) + "\n"


def valu_rows(csv_path: str, simds: int = 1024, clock_ghz: float = 2.4):
    """Per kernel, averaged over its dispatches, from a rocprofv3 --pmc counter CSV with
    SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_THREAD_CYCLES_VALU (and optionally SQ_INSTS_LDS,
    SQ_INSTS_SALU, SQ_WAVES): wave-level VALU instructions per launch, the VALU lane utilisation
    SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU), and the time the VALU instructions need at
    one wave64 instruction per 4 cycles on every SIMD (the issue floor of the launch)."""
    import collections
    import csv
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(csv_path)):
        acc[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    rows = []
    for k, c in acc.items():
        if "SQ_INSTS_VALU" not in c:
            continue
        avg = {n: sum(v) / len(v) for n, v in c.items()}
        util = avg["SQ_THREAD_CYCLES_VALU"] / (64.0 * avg["SQ_ACTIVE_INST_VALU"]) if avg.get("SQ_ACTIVE_INST_VALU") else None
        floor_ms = avg["SQ_INSTS_VALU"] * 4.0 / simds / (clock_ghz * 1e6)
        rows.append((k, len(c["SQ_INSTS_VALU"]), avg, util, floor_ms))
    return sorted(rows, key=lambda r: -r[2]["SQ_INSTS_VALU"])


def valu_markdown(csv_path: str, title: str, command: str, note: str) -> str:
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "", note, "",
           "| kernel | launches | VALU instr / launch | LDS instr / launch | SALU instr / launch | VALU lane utilisation | VALU issue floor (ms) |",
           "|---|---|---|---|---|---|---|"]
    for k, n, avg, util, floor_ms in valu_rows(csv_path):
        lds = avg.get("SQ_INSTS_LDS")
        salu = avg.get("SQ_INSTS_SALU")
        out.append(f"| {k} | {n} | {avg['SQ_INSTS_VALU']:.3e} | " + (f"{lds:.3e}" if lds is not None else "-") + " | "
                   + (f"{salu:.3e}" if salu is not None else "-") + " | " + (f"{100 * util:.1f} %" if util else "-")
                   + f" | {floor_ms:.3f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    if sys.argv[1] == "valu":
        src, title, command, note, dest = sys.argv[2:7]
        open(dest, "w").write(valu_markdown(src, title, command, note))
    else:
        db, title, command, note, dest = sys.argv[1:6]
        open(dest, "w").write(markdown(db, title, command, note))
