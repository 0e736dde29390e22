"""Turns a rocprofv3 --stats kernel_stats.csv into the short text summary kept in profiles/.

usage: python profiles/make_summary.py <kernel_stats.csv> <out.txt> <title> <command> [note]
"""
import csv
import sys


def main():
    src, out, title, command = sys.argv[1:5]
    note = sys.argv[5] if len(sys.argv) > 5 else ""
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


if __name__ == "__main__":
    main()
