"""Turns rocprofv3 output into the short text summaries kept under profiles/.

usage:
  python -m paper_2412_03898_amd.profsum stats <kernel_stats.csv> <out.txt> <title> <command> [note]
  python -m paper_2412_03898_amd.profsum counters <out.txt> <title> <note> <command1> <csv1> [<command2> <csv2> ...]

  python -m paper_2412_03898_amd.profsum traffic <out.json> <kernel> <workload> <fetch.csv> <write.csv> <fetch_scale> <write_scale> <fetch_cmd> <write_cmd> <source>...
  python -m paper_2412_03898_amd.profsum sq <out.json> <kernel> <workload> <counter.csv> <cmd> <source>...
  (traffic and sq take an optional first argument --skip=K: leave out the kernel's first K dispatches)

`traffic` records the HBM bytes per dispatch of one kernel (dispatches whose name
contains <kernel>), scaled by the copy-calibration factors, together with a
SHA-256 over the source files the kernel is built from: bench.py reports the
figure only while those sources are unchanged.

Counter tables keep only the library's own kernels (names containing "sb::")
and the runtime's copy kernel used to calibrate the memory counters.

`sq` records the mean per dispatch of every counter in one --pmc run for one
kernel (for instance SQ_INSTS_VALU, the issued vector instructions), with the
same source digest.

`stats` tabulates a --kernel-trace --stats summary; `counters` averages each
counter of one or more --pmc counter_collection.csv files per kernel and lists
the commands that produced them.
"""
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


_C_LIKE = (".hip", ".hpp", ".h", ".c", ".cpp")


def code_text(rel: str, data: bytes) -> bytes:
    """The part of a source file that the digest covers: for C-like files the code with
    comments removed and whitespace runs collapsed (editing a comment does not change
    what the kernel does), else the file as it is."""
    if not rel.endswith(_C_LIKE):
        return data
    text = data.decode("utf-8", errors="replace")
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split()).encode()


def source_digest(paths, read=None):
    """SHA-256 over the code of the named files (paths relative to the repository root),
    in order.  `read(rel) -> bytes` supplies the contents (default: the working tree)."""
    h = hashlib.sha256()
    for rel in paths:
        if read is None:
            with open(os.path.join(ROOT, rel), "rb") as f:
                data = f.read()
        else:
            data = read(rel)
        h.update(rel.encode() + b"\0" + code_text(rel, data))
    return h.hexdigest()


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


def _dispatch_values(path, kernel, counter, skip):
    """Values of `counter` for the dispatches of `kernel` in dispatch order, without the
    first `skip` of them (for instance a launch that prepares the measured data)."""
    rows = [r for r in csv.DictReader(open(path)) if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in rows[skip:]]


def traffic(out, kernel, workload, fetch_csv, write_csv, fetch_scale, write_scale, fetch_cmd, write_cmd,
            sources, skip=0):
    def mean(path, counter):
        v = _dispatch_values(path, kernel, counter, skip)
        if not v:
            raise SystemExit(f"no {counter} dispatch of {kernel} in {path}")
        return sum(v) / len(v), len(v)
    fk, nf = mean(fetch_csv, "FETCH_SIZE")
    wk, nw = mean(write_csv, "WRITE_SIZE")
    rec = {"kernel": kernel, "workload": workload, "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
           "dispatches": [nf, nw], "fetch_scale": float(fetch_scale), "write_scale": float(write_scale),
           "bytes_per_launch": round(float(fetch_scale) * fk * 1024 + float(write_scale) * wk * 1024),
           "skipped_first_dispatches": skip,
           "commands": [fetch_cmd, write_cmd], "sources": sources, "source_sha256": source_digest(sources)}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def sq(out, kernel, workload, csv_path, command, sources, skip=0):
    names = sorted({r["Counter_Name"] for r in csv.DictReader(open(csv_path)) if kernel in r["Kernel_Name"]})
    agg = {c: _dispatch_values(csv_path, kernel, c, skip) for c in names}
    agg = {c: v for c, v in agg.items() if v}
    if not agg:
        raise SystemExit(f"no dispatch of {kernel} in {csv_path}")
    rec = {"kernel": kernel, "workload": workload,
           "counters": {k: round(sum(v) / len(v), 1) for k, v in sorted(agg.items())},
           "dispatches": max(len(v) for v in agg.values()), "skipped_first_dispatches": skip,
           "command": command, "sources": sources, "source_sha256": source_digest(sources)}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def _record_for(suffix: str, kernel: str, workload: str):
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(suffix):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            rec = json.load(f)
        if rec.get("kernel") != kernel or rec.get("workload") != workload:
            continue
        try:
            if source_digest(rec["sources"]) != rec["source_sha256"]:
                return None
        except OSError:
            return None
        return rec
    return None


def sq_for(kernel: str, workload: str, counter: str = "SQ_INSTS_VALU"):
    """Mean per dispatch of an SQ counter recorded for (kernel, workload) under profiles/,
    or None when there is no record or the kernel's sources changed since."""
    rec = _record_for("_sq.json", kernel, workload)
    return None if rec is None else rec["counters"].get(counter)


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch recorded for (kernel, workload) under profiles/, or None when
    there is no record or the kernel's sources changed since the counters were taken."""
    rec = _record_for("_traffic.json", kernel, workload)
    return None if rec is None else rec["bytes_per_launch"]


def main():
    mode = sys.argv[1]
    if mode == "stats":
        stats(*sys.argv[2:])
    elif mode == "counters":
        out, title, note = sys.argv[2:5]
        rest = sys.argv[5:]
        counters(out, title, note, list(zip(rest[0::2], rest[1::2])))
    elif mode in ("traffic", "sq"):
        a = sys.argv[2:]
        skip = 0
        if a and a[0].startswith("--skip="):
            skip = int(a[0].split("=", 1)[1])
            a = a[1:]
        if mode == "traffic":
            traffic(*a[:9], sources=a[9:], skip=skip)
        else:
            sq(*a[:5], sources=a[5:], skip=skip)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main()
