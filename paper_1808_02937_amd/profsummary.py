"""Summarise a rocprofv3 --kernel-trace --stats CSV run into short markdown tables.

usage: python -m paper_1808_02937_amd.profsummary <dir-with-*_kernel_stats.csv> "<command>" > out.md
"""
import csv
import glob
import os
import re
import sys
from collections import defaultdict


def short(name):
    name = name.replace("fde::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)


def main():
    d, cmd = sys.argv[1], sys.argv[2]
    stats = glob.glob(os.path.join(d, "*_kernel_stats.csv"))[0]
    trace = glob.glob(os.path.join(d, "*_kernel_trace.csv"))[0]
    rows = list(csv.DictReader(open(stats)))
    print(f"command: `{cmd}`\n")
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---|---|---|---|")
    for r in rows[:15]:
        print(f"| {short(r['Name'])} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    # level launches of the H-LU (one kernel per level of the schedule) and H-solve launches
    tr = list(csv.DictReader(open(trace)))
    by = defaultdict(list)
    for t in tr:
        name = short(t["Kernel_Name"])
        if name.startswith("k_level") or name.startswith("k_hsolve"):
            dur = (int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) / 1e3
            by[(name, t["Grid_Size_X"] if name.startswith("k_hsolve") else "per level")].append(dur)
    if by:
        print("\n| kernel | grid x (threads) | launches | avg us | max us | total ms |")
        print("|---|---|---|---|---|---|")
        for (k, g), v in sorted(by.items()):
            print(f"| {k} | {g} | {len(v)} | {sum(v) / len(v):.1f} | {max(v):.1f} | {sum(v) / 1e3:.2f} |")

if __name__ == "__main__":
    main()
