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


if __name__ == "__main__":
    db, title, command, note, dest = sys.argv[1:6]
    open(dest, "w").write(markdown(db, title, command, note))
