"""Summarise a rocprofv3 --kernel-trace --stats CSV run into a short markdown table.

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
    # split launches of the interpreter by grid size (batched H-LU: grid = number of operators, one long launch)
    tr = list(csv.DictReader(open(trace)))
    by = defaultdict(list)
    for t in tr:
        if "k_interp" in t["Kernel_Name"]:
            dur = (int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) / 1e6
            kind = "H-LU" if dur > 200 else "H-solve"
            by[(short(t["Kernel_Name"]), kind, t["Grid_Size_X"])].append(dur)
    if by:
        print("\n| interpreter launch | kind | grid x (threads) | launches | avg ms |")
        print("|---|---|---|---|---|")
        for (k, kind, g), v in sorted(by.items()):
            print(f"| {k} | {kind} | {g} | {len(v)} | {sum(v) / len(v):.3f} |")


if __name__ == "__main__":
    main()
