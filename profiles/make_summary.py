"""Turns rocprofv3 output into the short text summaries kept next to this script.

usage:
  python profiles/make_summary.py stats <kernel_stats.csv> <out.txt> <title> <command> [note]
  python profiles/make_summary.py counters <out.txt> <title> <note> <command1> <csv1> [<command2> <csv2> ...]

Counter tables keep only the library's own kernels (names containing "sb::")
and the runtime's copy kernel used to calibrate the memory counters.

`stats` tabulates a --kernel-trace --stats summary; `counters` averages each
counter of one or more --pmc counter_collection.csv files per kernel and lists
the commands that produced them.
"""
import collections
import csv
import sys


def stats(src, out, title, command, note=""):
    rows = list(csv.DictReader(open(src)))
    lines = [title, "", "Command (MI355X, from the repository root):", "  " + command, ""]
    if note:
        lines += [note, ""]
    lines.append(f"{'kernel':<62} {'calls':>6} {'avg_us':>11} {'min_us':>11} {'max_us':>11} {'pct':>7}")
    for r in rows:
        lines.append(f"{r['Name'][:60]:<62} {r['Calls']:>6} {float(r['AverageNs']) / 1e3:>11.2f} "
                     f"{float(r['MinNs']) / 1e3:>11.2f} {float(r['MaxNs']) / 1e3:>11.2f} "
                     f"{float(r['Percentage']):>7.2f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(out, title, note, pairs):
    lines = [title, "", note, "", "Commands (MI355X, from the repository root):"]
    agg = collections.defaultdict(list)
    order = []
    for command, src in pairs:
        lines.append("  " + command)
        for r in csv.DictReader(open(src)):
            if "sb::" not in r["Kernel_Name"] and "copyBuffer" not in r["Kernel_Name"]:
                continue
            key = (r["Kernel_Name"], r["Counter_Name"])
            if key not in agg:
                order.append(key)
            agg[key].append(float(r["Counter_Value"]))
    lines += ["", f"{'kernel':<62} {'counter':<22} {'dispatches':>10} {'mean per dispatch':>18}"]
    for key in sorted(order, key=lambda k: (k[0], k[1])):
        v = agg[key]
        lines.append(f"{key[0][:60]:<62} {key[1]:<22} {len(v):>10} {sum(v) / len(v):>18.1f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    mode = sys.argv[1]
    if mode == "stats":
        stats(*sys.argv[2:])
    elif mode == "counters":
        out, title, note = sys.argv[2:5]
        rest = sys.argv[5:]
        counters(out, title, note, list(zip(rest[0::2], rest[1::2])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main()
