"""Summarise rocprofv3 outputs (kernel-trace SQLite/CSV, PMC CSV) into the
short text tables kept in this folder.

    python profiles/summarize.py trace <results.db | kernel_stats.csv>
    python profiles/summarize.py pmc <counter_collection.csv> [...]
"""
import csv
import sqlite3
import sys
from collections import defaultdict


def trace(path):
    agg = defaultdict(list)
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        names = dict(con.execute("select id, kernel_name from rocpd_info_kernel_symbol"))
        for k, s, e in con.execute("select kernel_id, start, end from rocpd_kernel_dispatch"):
            agg[names.get(k, str(k))].append((e - s) / 1e6)
    else:
        for row in csv.DictReader(open(path)):
            if "Kernel_Name" in row:
                agg[row["Kernel_Name"]].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e6)
    print(f"{'kernel':58s} {'calls':>5s} {'avg_ms':>9s} {'total_ms':>9s}")
    for k, v in sorted(agg.items(), key=lambda x: -sum(x[1])):
        print(f"{k.split('(')[0][:58]:58s} {len(v):5d} {sum(v) / len(v):9.3f} {sum(v):9.2f}")


def pmc(paths):
    agg = defaultdict(lambda: defaultdict(float))
    calls = defaultdict(set)
    for path in paths:
        for row in csv.DictReader(open(path)):
            k = row.get("Kernel_Name", "?").split("(")[0]
            agg[k][row["Counter_Name"]] += float(row["Counter_Value"])
            calls[k].add(row.get("Dispatch_Id", ""))
    for k, cs in agg.items():
        n = max(len(calls[k]), 1)
        print(f"{k[:70]}  (dispatches: {n}; values per dispatch)")
        for c, v in sorted(cs.items()):
            print(f"    {c:28s} {v / n:16.4g}")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    else:
        pmc(sys.argv[2:])
